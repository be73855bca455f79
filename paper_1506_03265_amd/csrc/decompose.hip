// CLUSTER(G, tau) of Algorithm 1 (Section 3 of arXiv:1506.03265) on gfx950.
//
// Design
// ------
// One device job decomposes a batch of graphs (a single graph is a batch of
// one).  Every graph runs its own state machine
//
//   SELECT -> RELAX* -> [NEXT -> RELAX*]* -> ASSIGN -> RMAX -> COMPACT -> SELECT ...
//                                                              -> SINGLE -> DONE
//
// and all graphs advance in lock step through "sweeps": in one sweep every
// graph contributes the items of the list its phase works on (uncovered
// nodes, frontier, blocked nodes or newly covered nodes), the items of all
// graphs form one index space, and every wave of the grid takes 64 of them.
// Between sweeps one workgroup runs the per-graph control step (one thread
// per graph), which applies Algorithm 1's decisions: coverage test, Delta
// doubling, stage end, termination.
//
// Node state is one u64 key per node: (growth distance << 32) | center id,
// ~0 when unset.  An offer (d_u + w, c_u) is applied with a 64-bit atomicMin,
// so concurrent offers resolve to the lexicographic minimum and the fixpoint
// of a growth level is unique whatever the order of relaxations; no step
// synchronisation is needed inside a level.  Nodes assigned in earlier
// stages keep key (0, cluster) and are sources of later stages (the effect of
// Procedure Contract); no contracted graph is built.
//
// Lists (per graph, each of the graph's node count; all are node ids local to
// the graph):
//   U[2]          uncovered nodes (current / compacted)
//   pool[3]       frontier (current, next) and blocked list, roles rotate
//   C             nodes covered in the current stage
// A node is pushed on the next frontier when its key improves (once per sweep,
// deduplicated by a sweep stamp), on C when its key first becomes finite, and
// on the blocked list when its scan stopped at an arc heavier than
// Delta - d_u (once per level, level stamp).  At a level's fixpoint every arc
// from a reached node into an unreached one is such a blocked arc, so:
//   - the smallest distance at which a new node becomes reachable is the
//     minimum over blocked arcs into unreached nodes of d_u + w (NEXT), and
//     Delta doublings below it cannot change anything, so they are applied
//     without growth;
//   - the blocked list is exactly the set of nodes to rescan after Delta grows,
//     and after the stage it is the set of assigned nodes adjacent to the
//     remaining uncovered nodes, i.e. the sources of the next stage.
//
// Drivers: a persistent cooperative kernel that alternates sweep and control
// with grid barriers (one launch per job), or host-driven launches of a sweep
// kernel and a control kernel (the host polls a done flag).  Both run the
// same device code.

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "common.h"

namespace {

enum Phase : uint32_t {
  PH_START = 0,
  PH_SELECT = 1,
  PH_RELAX = 2,
  PH_NEXT = 3,
  PH_ASSIGN = 4,
  PH_RMAX = 5,
  PH_COMPACT = 6,
  PH_SINGLE = 7,
  PH_DONE = 8,
};

struct GDesc {
  const int32_t *row_ptr;
  const uint64_t *arcs;
  int32_t *cluster;
  uint64_t *D;
  int64_t off;       // offset of this graph in node-indexed workspace arrays
  double K;          // (gamma * tau) * log2(n)
  uint64_t seed;
  int32_t n;
  uint32_t stop;     // ceil(8 tau log2 n)
  uint32_t delta0;
  uint32_t pad;
};

struct GState {
  // control-owned
  uint32_t phase, stage, delta, level_id;
  uint64_t T;
  uint32_t nU, ucur;
  uint32_t fcur, fnxt, blk;
  int32_t status;
  uint32_t levels, sweeps, centers_total, singletons;
  // sweep counters
  uint32_t cnt[3];
  uint32_t cntU[2];
  uint32_t cntC;
  uint32_t centers;
  uint64_t next;
  uint64_t radius;
  uint64_t arcs;
};

struct Ctl {
  uint32_t sweep_id;  // stamp of the current sweep (>= 1)
  uint32_t done;      // 1 when every graph is DONE
  uint32_t total;     // items of the current sweep
  uint32_t error;     // first error status (as positive code) or 0
  uint32_t iterations;
  uint32_t timeout;   // barrier wait gave up
  unsigned long long arcs;  // arcs read by relaxation (diagnostic)
  unsigned long long t_start;   // wall clock at the first control step
  unsigned long long t_limit;   // ticks after which the job stops with a timeout
  CldBarrier bar;
};

struct Job {
  const GDesc *desc;
  GState *st;
  Ctl *ctl;
  uint32_t *seg;     // G + 1 exclusive prefix of per-graph sweep items
  int32_t *log;      // G x CLDIAM_STAGE_LOG x 4
  uint64_t *key;
  uint64_t *R;
  uint32_t *fstamp;
  uint32_t *bstamp;
  int32_t *pool[3];
  int32_t *U[2];
  int32_t *C;
  int32_t G;
};

constexpr int kThreads = 256;
constexpr int kJobSeconds = 60;  // device-side limit of one decomposition job

// ------------------------------------------------------------- control --

__device__ uint32_t items_of(const GState &s) {
  switch (s.phase) {
    case PH_SELECT: case PH_COMPACT: case PH_SINGLE: return s.cntU[s.ucur];
    case PH_RELAX: return s.cnt[s.fcur];
    case PH_NEXT: return s.cnt[s.blk];
    case PH_ASSIGN: case PH_RMAX: return s.cntC;
    default: return 0;
  }
}

__device__ void fail(GState &s, Ctl *ctl, int status) {
  s.status = status;
  s.phase = PH_DONE;
  atomicCAS(&ctl->error, 0u, (uint32_t)(-status));
}

__device__ void begin_stage(const GDesc &d, GState &s, Ctl *ctl) {
  if (s.nU == 0 || s.nU < d.stop || d.n < 2) {
    s.phase = PH_SINGLE;
    return;
  }
  if (s.stage >= CLDIAM_MAX_STAGES) {
    fail(s, ctl, CLDIAM_ESTAGES);
    return;
  }
  double p = d.K / (double)s.nU;
  s.T = p >= 1.0 ? ((uint64_t)1 << 32) : (uint64_t)floor(p * 4294967296.0);
  s.centers = 0;
  s.cntC = 0;
  s.phase = PH_SELECT;
}

// Per-graph transition after a sweep of its current phase.
__device__ void control_graph(const Job &job, int g, uint32_t sweep_id) {
  const GDesc &d = job.desc[g];
  GState &s = job.st[g];
  switch (s.phase) {
    case PH_START:
      s.delta = d.delta0;
      s.stage = 0;
      s.nU = (uint32_t)d.n;
      s.cntU[0] = (uint32_t)d.n;
      s.ucur = 0;
      s.fcur = 0; s.fnxt = 1; s.blk = 2;
      s.cnt[0] = s.cnt[1] = s.cnt[2] = 0;
      if ((uint64_t)s.delta > CLD_DELTA_MAX) { fail(s, job.ctl, CLDIAM_EOVERFLOW); break; }
      begin_stage(d, s, job.ctl);
      break;
    case PH_SELECT:
      // frontier = sources from the previous stage + the new centers
      s.centers_total += s.centers;
      s.level_id = sweep_id;
      s.levels++;
      s.phase = PH_RELAX;
      break;
    case PH_RELAX:
      s.sweeps++;
      if (s.cnt[s.fnxt] > 0) {
        uint32_t t = s.fcur; s.fcur = s.fnxt; s.fnxt = t;
        s.cnt[s.fnxt] = 0;
      } else {
        s.cnt[s.fcur] = 0;
        if (2ull * s.cntC >= (uint64_t)s.nU) s.phase = PH_ASSIGN;
        else { s.next = CLD_INF64; s.phase = PH_NEXT; }
      }
      break;
    case PH_NEXT:
      if (s.next == CLD_INF64) {
        s.phase = PH_ASSIGN;
      } else {
        uint64_t dl = s.delta;
        do {
          if (2 * dl > CLD_DELTA_MAX) { fail(s, job.ctl, CLDIAM_EOVERFLOW); return; }
          dl *= 2;
          s.levels++;
        } while (dl < s.next);
        s.delta = (uint32_t)dl;
        // rescan the blocked nodes at the new Delta; fresh blocked list
        uint32_t t = s.fcur; s.fcur = s.blk; s.blk = t;
        s.cnt[s.blk] = 0;
        s.level_id = sweep_id;
        s.phase = PH_RELAX;
      }
      break;
    case PH_ASSIGN:
      s.phase = PH_RMAX;
      break;
    case PH_RMAX: {
      s.cntU[s.ucur ^ 1] = 0;
      s.phase = PH_COMPACT;
      break;
    }
    case PH_COMPACT: {
      if (s.stage < CLDIAM_STAGE_LOG) {
        int32_t *lg = job.log + ((size_t)g * CLDIAM_STAGE_LOG + s.stage) * 4;
        lg[0] = (int32_t)s.nU; lg[1] = (int32_t)s.centers; lg[2] = (int32_t)s.cntC; lg[3] = (int32_t)s.delta;
      }
      s.ucur ^= 1;
      s.nU = s.cntU[s.ucur];
      s.stage++;
      // sources of the next stage: the blocked list of the last level
      uint32_t t = s.fcur; s.fcur = s.blk; s.blk = t;
      s.cnt[s.blk] = 0;
      s.cnt[s.fnxt] = 0;
      begin_stage(d, s, job.ctl);
      break;
    }
    case PH_SINGLE:
      s.singletons = s.nU;
      s.phase = PH_DONE;
      break;
    default:
      break;
  }
}

// One workgroup: control of every graph, then the next sweep's index space.
__device__ void control_block(const Job &job) {
  __shared__ uint32_t scan[kThreads];
  __shared__ uint32_t carry, alldone;
  Ctl *ctl = job.ctl;
  uint32_t sweep_id = ctl->sweep_id + 1;
  if (threadIdx.x == 0) {
    carry = 0;
    alldone = 1;
    const unsigned long long now = wall_clock64();
    if (ctl->iterations == 0) ctl->t_start = now;
    else if (now - ctl->t_start > ctl->t_limit && ctl->error == 0) atomicCAS(&ctl->error, 0u, (uint32_t)(-CLDIAM_ETIMEOUT));
  }
  __syncthreads();
  for (int base = 0; base < job.G; base += kThreads) {
    int g = base + (int)threadIdx.x;
    uint32_t items = 0;
    if (g < job.G) {
      if (ctl->error == 0 || job.st[g].phase == PH_DONE) control_graph(job, g, sweep_id);
      if (ctl->error != 0 && job.st[g].phase != PH_DONE) job.st[g].phase = PH_DONE;
      items = items_of(job.st[g]);
      if (job.st[g].phase != PH_DONE) atomicAnd(&alldone, 0u);
    }
    scan[threadIdx.x] = items;
    __syncthreads();
    for (int o = 1; o < kThreads; o <<= 1) {
      uint32_t x = threadIdx.x >= (unsigned)o ? scan[threadIdx.x - o] : 0;
      __syncthreads();
      scan[threadIdx.x] += x;
      __syncthreads();
    }
    if (g < job.G) job.seg[g] = carry + scan[threadIdx.x] - items;
    __syncthreads();
    if (threadIdx.x == kThreads - 1) carry += scan[kThreads - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    job.seg[job.G] = carry;
    ctl->total = carry;
    ctl->sweep_id = sweep_id;
    ctl->iterations++;
    ctl->done = alldone;
  }
}

// --------------------------------------------------------------- sweeps --

__device__ __forceinline__ void push(const Job &job, int32_t *list, uint32_t *counter, int64_t off, bool pred,
                                     int32_t v) {
  uint32_t slot = cld_wave_reserve(pred, counter);
  if (pred) list[off + slot] = v;
}

// RELAX: scan the light prefix of u's row (w <= Delta - d_u) and offer
// (d_u + w, c_u) to every neighbour.
__device__ uint32_t relax_item(const Job &job, const GDesc &d, GState &s, uint32_t it, int32_t u) {
  const int64_t off = d.off;
  const uint32_t fnxt = s.fnxt, blk = s.blk, level_id = s.level_id;
  int32_t *const fl = job.pool[fnxt];
  int32_t *const bl = job.pool[blk];
  const uint64_t ku = job.key[off + u];
  const uint32_t lim = s.delta - (uint32_t)(ku >> 32);
  int32_t a = d.row_ptr[u];
  const int32_t a1 = d.row_ptr[u + 1];
  bool blocked = false;
  uint32_t scanned = 0;
  for (; a < a1; ++a) {
    const uint64_t arc = d.arcs[a];
    const uint32_t w = (uint32_t)(arc >> 32);
    if (w > lim) { blocked = true; break; }
    ++scanned;
    const int64_t gv = off + (int32_t)(uint32_t)arc;
    const uint64_t cand = ku + ((uint64_t)w << 32);
    bool newly = false, front = false;
    if (cand < job.key[gv]) {
      const uint64_t old = atomicMin((unsigned long long *)&job.key[gv], (unsigned long long)cand);
      if (cand < old) {
        newly = (old == CLD_INF64);
        if (job.fstamp[gv] != it) front = atomicExch(&job.fstamp[gv], it) != it;
      }
    }
    const int32_t v = (int32_t)(uint32_t)arc;
    push(job, job.C, &s.cntC, off, newly, v);
    push(job, fl, &s.cnt[fnxt], off, front, v);
  }
  bool addb = false;
  if (blocked && job.bstamp[off + u] != level_id) addb = atomicExch(&job.bstamp[off + u], level_id) != level_id;
  push(job, bl, &s.cnt[blk], off, addb, u);
  return scanned;
}

// NEXT: smallest d_u + w over arcs from blocked node u to unreached nodes.
__device__ void next_item(const Job &job, const GDesc &d, GState &s, int32_t u) {
  const int64_t off = d.off;
  const uint64_t ku = job.key[off + u];
  const uint32_t du = (uint32_t)(ku >> 32);
  const uint32_t lim = s.delta - du;
  const int32_t a0 = d.row_ptr[u];
  uint64_t best = CLD_INF64;
  for (int32_t a = d.row_ptr[u + 1] - 1; a >= a0; --a) {
    const uint64_t arc = d.arcs[a];
    const uint32_t w = (uint32_t)(arc >> 32);
    if (w <= lim) break;
    if (job.key[off + (int32_t)(uint32_t)arc] == CLD_INF64) {
      const uint64_t c = (uint64_t)du + w;
      best = c < best ? c : best;
    }
  }
  if (best != CLD_INF64) atomicMin((unsigned long long *)&s.next, (unsigned long long)best);
}

__device__ uint32_t process(const Job &job, int g, uint32_t idx, uint32_t it) {
  const GDesc &d = job.desc[g];
  GState &s = job.st[g];
  const int64_t off = d.off;
  uint32_t scanned = 0;
  switch (s.phase) {
    case PH_SELECT: {
      const int32_t v = job.U[s.ucur][off + idx];
      const uint32_t x0 = cld_philox_word0((uint32_t)v, s.stage, 0u, 0u, (uint32_t)d.seed, (uint32_t)(d.seed >> 32));
      const bool c = (uint64_t)x0 < s.T;
      if (c) job.key[off + v] = (uint64_t)(uint32_t)v;
      push(job, job.pool[s.fcur], &s.cnt[s.fcur], off, c, v);
      push(job, job.C, &s.cntC, off, c, v);
      unsigned long long m = __ballot(c);
      if (m && cld_lane() == __ffsll((long long)m) - 1) atomicAdd(&s.centers, (uint32_t)__popcll(m));
      break;
    }
    case PH_RELAX:
      scanned = relax_item(job, d, s, it, job.pool[s.fcur][off + idx]);
      break;
    case PH_NEXT:
      next_item(job, d, s, job.pool[s.blk][off + idx]);
      break;
    case PH_ASSIGN: {
      const int32_t v = job.C[off + idx];
      const uint64_t k = job.key[off + v];
      const uint32_t c = (uint32_t)k;
      const uint64_t Dv = (k >> 32) + job.R[off + c];
      d.cluster[v] = (int32_t)c;
      d.D[v] = Dv;
      if (Dv > s.radius) atomicMax((unsigned long long *)&s.radius, (unsigned long long)Dv);
      break;
    }
    case PH_RMAX: {
      const int32_t v = job.C[off + idx];
      const uint32_t c = (uint32_t)job.key[off + v];
      const uint64_t Dv = d.D[v];
      uint64_t *r = &job.R[off + c];
      if (Dv > *r) atomicMax((unsigned long long *)r, (unsigned long long)Dv);
      job.key[off + v] = (uint64_t)c;
      break;
    }
    case PH_COMPACT: {
      const int32_t v = job.U[s.ucur][off + idx];
      const bool keep = job.key[off + v] == CLD_INF64;
      push(job, job.U[s.ucur ^ 1], &s.cntU[s.ucur ^ 1], off, keep, v);
      break;
    }
    case PH_SINGLE: {
      const int32_t v = job.U[s.ucur][off + idx];
      d.cluster[v] = v;
      d.D[v] = 0;
      break;
    }
    default:
      break;
  }
  return scanned;
}

// Item index -> graph (largest g with seg[g] <= i).
__device__ __forceinline__ int graph_of(const Job &job, uint32_t i) {
  int lo = 0, hi = job.G - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (job.seg[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Logical wave id with consecutive ids on one XCD (blocks are dealt to the 8
// XCDs round-robin), so neighbouring chunks of a list share an L2.
__device__ __forceinline__ uint32_t logical_block(uint32_t b, uint32_t nb) {
  if (nb % 8u) return b;
  return (b & 7u) * (nb >> 3) + (b >> 3);
}

__device__ void sweep(const Job &job, uint32_t block, uint32_t nblocks) {
  const uint32_t total = job.ctl->total;
  const uint32_t it = job.ctl->sweep_id;
  const uint32_t waves_per_block = blockDim.x >> 6;
  const uint32_t wave = logical_block(block, nblocks) * waves_per_block + (threadIdx.x >> 6);
  const uint32_t nwaves = nblocks * waves_per_block;
  uint32_t scanned = 0;
  for (uint32_t chunk = wave; (uint64_t)chunk * 64 < total; chunk += nwaves) {
    const uint32_t i = chunk * 64 + (uint32_t)cld_lane();
    int g = i < total ? graph_of(job, i) : 0x7fffffff;
    for (;;) {
      int gmin = g;
      for (int o = 32; o >= 1; o >>= 1) {
        int x = __shfl_xor(gmin, o);
        gmin = x < gmin ? x : gmin;
      }
      gmin = __builtin_amdgcn_readfirstlane(gmin);
      if (gmin == 0x7fffffff) break;
      if (g == gmin) {
        scanned += process(job, gmin, i - job.seg[gmin], it);
        g = 0x7fffffff;
      }
    }
  }
  for (int o = 32; o >= 1; o >>= 1) scanned += __shfl_xor(scanned, o);
  if (cld_lane() == 0 && scanned) atomicAdd(&job.ctl->arcs, (unsigned long long)scanned);
}

// ---------------------------------------------------------------- kernels --

__global__ void __launch_bounds__(kThreads) k_init(Job job, int64_t total_n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total_n; i += stride) {
    job.key[i] = CLD_INF64;
    job.R[i] = 0;
    job.fstamp[i] = 0;
    job.bstamp[i] = 0;
  }
  // U[0] of each graph = 0..n-1
  for (int g = 0; g < job.G; ++g) {
    const GDesc &d = job.desc[g];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.n; i += stride)
      job.U[0][d.off + i] = (int32_t)i;
  }
}

__global__ void __launch_bounds__(kThreads) k_control(Job job) { control_block(job); }

__global__ void __launch_bounds__(kThreads) k_sweep(Job job) {
  if (job.ctl->done) return;
  sweep(job, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kThreads) k_persistent(Job job) {
  const uint32_t nb = gridDim.x;
  for (;;) {
    if (blockIdx.x == 0) control_block(job);
    if (!cld_grid_barrier(&job.ctl->bar, &job.ctl->timeout, nb)) return;
    if (job.ctl->done || job.ctl->timeout) return;
    sweep(job, blockIdx.x, nb);
    if (!cld_grid_barrier(&job.ctl->bar, &job.ctl->timeout, nb)) return;
  }
}

// ------------------------------------------------------------------- host --

struct Layout {
  GDesc *desc;
  GState *st;
  Ctl *ctl;
  uint32_t *seg;
  int32_t *log;
  uint64_t *key, *R;
  uint32_t *fstamp, *bstamp;
  int32_t *pool[3], *U[2], *C;
};

template <class A>
bool carve(A &a, int64_t N, int32_t G, Layout *L) {
  auto p_desc = a.template take<GDesc>(G);
  auto p_st = a.template take<GState>(G);
  auto p_ctl = a.template take<Ctl>(1);
  auto p_seg = a.template take<uint32_t>((size_t)G + 1);
  auto p_log = a.template take<int32_t>((size_t)G * CLDIAM_STAGE_LOG * 4);
  auto p_key = a.template take<uint64_t>(N);
  auto p_R = a.template take<uint64_t>(N);
  auto p_fs = a.template take<uint32_t>(N);
  auto p_bs = a.template take<uint32_t>(N);
  auto p0 = a.template take<int32_t>(N);
  auto p1 = a.template take<int32_t>(N);
  auto p2 = a.template take<int32_t>(N);
  auto u0 = a.template take<int32_t>(N);
  auto u1 = a.template take<int32_t>(N);
  auto c = a.template take<int32_t>(N);
  if (L) {
    *L = Layout{(GDesc *)p_desc, (GState *)p_st, (Ctl *)p_ctl, (uint32_t *)p_seg, (int32_t *)p_log,
                (uint64_t *)p_key, (uint64_t *)p_R, (uint32_t *)p_fs, (uint32_t *)p_bs,
                {(int32_t *)p0, (int32_t *)p1, (int32_t *)p2}, {(int32_t *)u0, (int32_t *)u1}, (int32_t *)c};
    return p_desc && c;
  }
  return true;
}

struct SizeArena {
  cld::Sizer s;
  template <class T>
  void *take(size_t n) { s.take<T>(n); return (void *)1; }
};

struct PtrArena {
  cld::Arena a;
  PtrArena(void *p, size_t c) : a(p, c) {}
  template <class T>
  void *take(size_t n) { return (void *)a.take<T>(n); }
};

thread_local Ctl *t_host_ctl = nullptr;

Ctl *host_ctl() {
  if (!t_host_ctl) {
    void *p = nullptr;
    if (hipHostMalloc(&p, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) return nullptr;
    t_host_ctl = (Ctl *)p;
  }
  return t_host_ctl;
}

}  // namespace

extern "C" size_t cldiam_decompose_workspace_size(int64_t total_n, int32_t num_graphs) {
  if (total_n < 1 || num_graphs < 1) return 0;
  SizeArena s;
  carve(s, total_n, num_graphs, nullptr);
  return s.s.used;
}

extern "C" int cldiam_decompose_batch(int32_t G, const cldiam_graph *gs, cldiam_stats *stats, int driver, void *ws,
                                      size_t ws_bytes, void *stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (G < 1 || !gs) { cld::set_error("decompose: num_graphs < 1 or no graphs"); return CLDIAM_EINVAL; }
  int64_t N = 0;
  std::vector<GDesc> desc(G);
  const double gamma = 4.0 * M_LN2;
  for (int g = 0; g < G; ++g) {
    const cldiam_graph &x = gs[g];
    if (x.n < 1 || x.m < 0 || x.m >= ((int64_t)1 << 31) || !x.d_row_ptr || (x.m && !x.d_arcs) || !x.d_cluster ||
        !x.d_D || x.params.tau < 1) {
      cld::set_error("decompose: invalid graph %d (n=%d m=%lld tau=%u)", g, x.n, (long long)x.m, x.params.tau);
      return CLDIAM_EINVAL;
    }
    GDesc &d = desc[g];
    memset(&d, 0, sizeof d);
    d.row_ptr = x.d_row_ptr;
    d.arcs = x.d_arcs;
    d.cluster = x.d_cluster;
    d.D = x.d_D;
    d.off = N;
    d.n = x.n;
    const double L = log2((double)x.n);
    d.K = gamma * x.params.tau * L;
    d.stop = (uint32_t)ceil(8.0 * x.params.tau * L);
    d.seed = x.params.seed;
    uint64_t d0 = x.params.delta0;
    if (d0 == 0) d0 = x.m > 0 ? x.weight_sum / (uint64_t)x.m : 1;
    if (d0 < 1) d0 = 1;
    if (d0 > CLD_DELTA_MAX) {
      cld::set_error("decompose: initial Delta %llu above 2^31 (graph %d)", (unsigned long long)d0, g);
      return CLDIAM_EOVERFLOW;
    }
    d.delta0 = (uint32_t)d0;
    N += x.n;
  }
  Layout L;
  PtrArena pa(ws, ws_bytes);
  if (!carve(pa, N, G, &L) || pa.a.used > ws_bytes) {
    cld::set_error("decompose: workspace of %zu bytes, %zu needed", ws_bytes, cldiam_decompose_workspace_size(N, G));
    return CLDIAM_ENOMEM;
  }
  Job job;
  job.desc = L.desc; job.st = L.st; job.ctl = L.ctl; job.seg = L.seg; job.log = L.log; job.key = L.key;
  job.R = L.R; job.fstamp = L.fstamp; job.bstamp = L.bstamp;
  for (int i = 0; i < 3; ++i) job.pool[i] = L.pool[i];
  job.U[0] = L.U[0]; job.U[1] = L.U[1]; job.C = L.C; job.G = G;

  CLD_HIP(hipMemcpyAsync(L.desc, desc.data(), sizeof(GDesc) * G, hipMemcpyHostToDevice, stream));
  CLD_HIP(hipMemsetAsync(L.st, 0, sizeof(GState) * G, stream));
  CLD_HIP(hipMemsetAsync(L.ctl, 0, sizeof(Ctl), stream));
  {
    int dev = 0, khz = 0;
    CLD_HIP(hipGetDevice(&dev));
    CLD_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) khz = 100000;
    const unsigned long long limit = (unsigned long long)khz * 1000ull * kJobSeconds;
    CLD_HIP(hipMemcpyAsync(&L.ctl->t_limit, &limit, sizeof limit, hipMemcpyHostToDevice, stream));
  }
  CLD_HIP(hipMemsetAsync(L.log, 0, sizeof(int32_t) * G * CLDIAM_STAGE_LOG * 4, stream));
  k_init<<<cld::blocks_for(N, kThreads, 8192), kThreads, 0, stream>>>(job, N);
  CLD_LAUNCH_CHECK("k_init");

  int blocks = 0;
  if (driver != CLDIAM_DRIVER_HOST) {
    int rc = cld::cooperative_blocks((const void *)k_persistent, kThreads, 4, &blocks);
    if (rc) return rc;
    if (blocks == 0 && driver == CLDIAM_DRIVER_PERSISTENT) {
      cld::set_error("decompose: device has no cooperative launch");
      return CLDIAM_EINVAL;
    }
  }
  Ctl *hc = host_ctl();
  if (!hc) { cld::set_error("decompose: pinned host buffer allocation failed"); return CLDIAM_EHIP; }
  if (blocks > 0) {
    void *args[] = {&job};
    CLD_HIP(hipLaunchCooperativeKernel((const void *)k_persistent, dim3(blocks), dim3(kThreads), args, 0, stream));
    CLD_HIP(hipMemcpyAsync(hc, L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    CLD_HIP(hipStreamSynchronize(stream));
    if (hc->timeout) { cld::set_error("decompose: grid barrier timed out"); return CLDIAM_ETIMEOUT; }
    if (!hc->done && !hc->error) { cld::set_error("decompose: persistent kernel ended early"); return CLDIAM_EHIP; }
  } else {
    const int sweep_blocks = 2048;
    int batch = 4;
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
      for (int i = 0; i < batch; ++i) {
        k_control<<<1, kThreads, 0, stream>>>(job);
        k_sweep<<<sweep_blocks, kThreads, 0, stream>>>(job);
      }
      CLD_LAUNCH_CHECK("k_sweep");
      CLD_HIP(hipMemcpyAsync(hc, L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
      CLD_HIP(hipStreamSynchronize(stream));
      if (hc->done) break;
      if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(kJobSeconds + 30)) {
        cld::set_error("decompose: host-driven job exceeded its time limit");
        return CLDIAM_ETIMEOUT;
      }
      if (batch < 64) batch *= 2;
    }
  }
  std::vector<GState> st(G);
  std::vector<int32_t> lg((size_t)G * CLDIAM_STAGE_LOG * 4);
  CLD_HIP(hipMemcpyAsync(st.data(), L.st, sizeof(GState) * G, hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipMemcpyAsync(lg.data(), L.log, sizeof(int32_t) * lg.size(), hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipStreamSynchronize(stream));
  int rc = CLDIAM_OK;
  for (int g = 0; g < G; ++g) {
    if (st[g].status != CLDIAM_OK && rc == CLDIAM_OK) {
      rc = st[g].status;
      cld::set_error("decompose: graph %d failed: %s", g, cldiam_strerror(rc));
    }
    if (!stats) continue;
    cldiam_stats &o = stats[g];
    memset(&o, 0, sizeof o);
    o.stages = (int32_t)st[g].stage;
    o.levels = (int32_t)st[g].levels;
    o.delta0 = desc[g].delta0;
    o.delta_end = st[g].delta;
    o.stop = (int32_t)desc[g].stop;
    o.num_clusters = (int32_t)(st[g].centers_total + st[g].singletons);
    o.singletons = (int32_t)st[g].singletons;
    o.sweeps = (int32_t)st[g].sweeps;
    o.radius = st[g].radius;
    o.arcs_scanned = (G == 1) ? hc->arcs : 0;
    o.status = st[g].status;
    for (int s = 0; s < CLDIAM_STAGE_LOG && s < o.stages; ++s) {
      const int32_t *l = &lg[((size_t)g * CLDIAM_STAGE_LOG + s) * 4];
      o.stage_uncovered[s] = l[0];
      o.stage_centers[s] = l[1];
      o.stage_covered[s] = l[2];
      o.stage_delta[s] = (uint32_t)l[3];
    }
  }
  if (rc == CLDIAM_OK && hc->error) {
    rc = -(int)hc->error;
    cld::set_error("decompose: device reported %s", cldiam_strerror(rc));
  }
  return rc;
}

extern "C" int cldiam_decompose(const cldiam_graph *g, cldiam_stats *stats, int driver, void *ws, size_t ws_bytes,
                                void *stream) {
  return cldiam_decompose_batch(1, g, stats, driver, ws, ws_bytes, stream);
}
