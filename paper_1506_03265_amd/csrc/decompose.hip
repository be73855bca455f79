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
// nodes, frontier, blocked nodes or newly covered nodes), each graph's items
// are cut into chunks (one per workgroup, or a few per workgroup on large
// dense graphs), workgroup b takes chunk b and further chunks go to whichever
// workgroup asks next.  Between sweeps one workgroup runs the per-graph
// control step (one thread per graph), which applies Algorithm 1's decisions:
// coverage test, Delta doubling, stage end, termination.
//
// A relaxation sweep takes only frontier nodes whose tentative distance lies
// in the current distance bucket (a narrower one for nodes with long rows)
// and keeps the others on the frontier, which orders the label-correcting
// growth like Delta-stepping without changing its fixpoint.
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
// Pushes are staged in LDS per workgroup and written out with one global
// reservation per list and flush; every list counter sits in its own 128-byte
// line, so the serialisation of same-address atomics stays off the critical
// path.
//
// Drivers: a persistent cooperative kernel that alternates sweep and control
// with grid barriers (one launch per job), or host-driven launches of a sweep
// kernel and a control kernel (the host polls a done flag).  Both run the
// same device code.

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <thread>
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
  PH_IDLE = 9,   // empty slot of a server job
  PH_COMMIT = 10,  // synchronous steps: publish the step's updates
  PH_MERGE = 11,   // synchronous steps: add the blocked list to the active list
  PH_C2_INIT = 12,      // CLUSTER2: fresh state for every node
  PH_C2_SELECT = 13,    // CLUSTER2: centers of iteration i with probability 2^i / n
  PH_C2_BOUNDARY = 14,  // CLUSTER2: Contract2's rescaled edges out of last iteration's clusters
  PH_C2_ASSIGN = 15,    // CLUSTER2: assignment, D = d + Delta2 (i - birth iteration)
  PH_PULL = 16,         // pull mode: unreached nodes take their best offer from reached neighbours
  PH_NEXT_PULL = 17,    // pull mode: NEXT computed from the unreached nodes' side
};

struct GDesc {
  const int64_t *row_ptr;   // n+1 arc offsets
  const uint64_t *arcs;
  int32_t *cluster;
  uint64_t *D;
  int64_t off;       // offset of this graph in node-indexed workspace arrays
  double K;          // (gamma * tau) * log2(n)
  uint64_t seed;
  int32_t n;
  uint32_t stop;     // ceil(8 tau log2 n)
  uint32_t delta0;
  uint32_t bucket;   // distance bucket width of RELAX sweeps; 0 = unbounded
  uint32_t variant;  // CLDIAM_VARIANT_*
  uint32_t step_cap; // synchronous steps: most steps per PartialGrowth call (0 = none)
  uint32_t c2_iters; // CLUSTER2: ceil(log2 n) iterations
  int32_t local_rounds;  // workgroup-local relaxation rounds per RELAX run
  int32_t row_shift;     // long rows use a bucket of width Delta >> row_shift; < 0 = none
  int32_t chunk_factor;  // RELAX / NEXT chunks per workgroup and sweep
  int32_t mid_deg;       // rows of more arcs are relaxed by one wave ("long rows")
  int32_t big_deg;       // rows of more arcs are relaxed by the whole workgroup
  uint32_t lq_cap;       // slots of the local relaxation queue used (at most kLocalCap)
  uint32_t pull_mode;    // CLDIAM_PULL_*: when new levels and stages pull from the unreached side
  uint32_t hub_deg;      // rows of more arcs are hub rows (kHubDegree x the average degree)
  uint64_t hub_min;      // more arcs than this in hub rows: a skewed, low-diameter graph
};

// Control-owned state of one graph.
struct GState {
  uint32_t phase, stage, delta, level_id;
  uint64_t T;
  uint32_t nU, ucur;
  uint32_t fcur, fnxt, blk;
  int32_t status;
  uint32_t levels, sweeps, centers_total, singletons;
  uint32_t theta;    // RELAX sweeps relax frontier nodes with tentative distance below theta
  uint32_t row_base; // ... and nodes of long rows only below row_limit(row_base)
  // synchronous steps
  uint32_t steps_call;  // steps of the current PartialGrowth call
  uint32_t fid;         // sweep id that stamped the current active list
  uint32_t after;       // phase after a MERGE sweep
  uint32_t c2;          // 1 while in CLUSTER2's iterations
  uint64_t rounds, updates;
  uint64_t radius1;     // CLUSTER2: R_CL of the preliminary CLUSTER run
  uint32_t pull;        // 1 once the graph grows new levels and stages by pulling (see PH_PULL)
  uint32_t pull_base;   // distance at which the current pulled level starts (its first bucket)
};

struct alignas(128) PadU32 {
  uint32_t v;
  uint32_t pad_[31];
};
struct alignas(128) PadU64 {
  unsigned long long v;
  uint32_t pad_[30];
};

// Counters written by sweeps, one 128-byte line each.
struct GCount {
  PadU32 cnt[3];   // pool lists
  PadU32 cntU[2];  // uncovered lists
  PadU32 cntC;     // covered list
  PadU32 centers;  // centers drawn in this stage
  PadU64 next;     // NEXT: smallest reach distance
  PadU64 radius;   // max D
  PadU32 fmin;     // RELAX: smallest tentative distance pushed on the next frontier
  PadU64 msgs;     // synchronous steps: offers sent
  PadU64 blk_arcs; // heavy arcs left on the rows of the blocked list (what a push rescan would read)
  PadU64 hub_arcs; // first SELECT (auto pull mode): arcs in hub rows
};

struct Ctl {
  uint32_t sweep_id;  // stamp of the current sweep (>= 1)
  uint32_t done;      // 1 when every graph is DONE
  uint32_t total;     // items of the current sweep
  uint32_t error;     // first error status (as positive code) or 0
  uint32_t iterations;
  uint32_t timeout;   // barrier wait gave up
  unsigned long long t_start;   // wall clock at the first control step
  unsigned long long t_limit;   // ticks after which the job stops with a timeout
  PadU64 arcs;                  // arcs read by relaxation (diagnostic)
  PadU32 cursor;                // chunks of the current sweep taken beyond the first nblocks
  PadU32 idle;                  // workgroups that have finished the current sweep
  CldBarrier bar;
};

struct Job {
  const GDesc *desc;
  GState *st;
  GCount *cn;
  Ctl *ctl;
  uint32_t *seg;     // [0, G]: exclusive prefix of per-graph work chunks; [G+1, 2G]: items per chunk;
                     // [2G+1, 3G]: items of the graph in this sweep
  int32_t *log;      // G x CLDIAM_STAGE_LOG x 4
  uint64_t *key;
  uint64_t *keyn;    // synchronous steps: state after the current step (key holds the state before it);
                     // otherwise, for long rows, the key of the row's last scan
  uint32_t *slim;    // with keyn: the light limit (Delta - d) of that scan; arcs up to it have been offered
  uint64_t *R;
  uint32_t *fstamp;
  uint32_t *bstamp;
  int32_t *pool[3];
  int32_t *U[2];
  int32_t *C;
  int32_t G;
  int32_t nblocks;        // workgroups of a sweep launch
  uint32_t *hmirror = nullptr;   // host-driven job: mapped pinned words {control steps done, done flag} that
                                 // the host polls while it queues steps (nullptr: not mirrored)
  uint32_t cutoff;        // a workgroup ends its local rounds once this many workgroups have finished the
                          // sweep (the rounds are optional: every improved node is on the next frontier)
};

constexpr int kThreads = 1024;        // control workgroup
constexpr int kSweepThreads = 1024;   // sweep workgroup
constexpr int kCuThreads = 1024;      // sweep threads resident per CU (16 waves at the sweep's register use)
constexpr int kStageCap = 4 * kSweepThreads;   // LDS staging slots per output list
constexpr int kLocalCap = 4 * kSweepThreads;   // LDS local-round queue slots
constexpr int kMidDeg = 32;       // default: rows above this degree are relaxed by one wave
constexpr int kBigDeg = 8192;     // default: rows above this degree are relaxed by the whole workgroup
constexpr int kMidCap = 2 * kSweepThreads;   // deferred wave rows per round
constexpr int kBigCap = kSweepThreads / 8;   // deferred workgroup rows per round
constexpr int kLocalRounds = 16;  // default local relaxation rounds per RELAX run
constexpr int kLocalCutoffPct = 75;    // default: local rounds end once this % of workgroups finished the sweep
constexpr int kDenseWaveRow = 128;     // default wave_row_min on graphs of more than kDenseDegree arcs per node
constexpr int kLocalRoundsDense = 2;   // ... on graphs with more than kDenseDegree arcs per node and
constexpr int kDenseDegree = 16;       // more than kDenseLarge nodes (none on smaller dense graphs)
constexpr int32_t kDenseLarge = 1 << 21;
constexpr int32_t kDenseChunks = 3;     // RELAX / NEXT chunks per workgroup on dense graphs
constexpr int32_t kRowShiftMin = 5;     // default long-row bucket: Delta >> shift, shift from the arc count
constexpr int32_t kRowShiftMax = 8;
constexpr uint32_t kSmallFrontier = 1u << 15;   // frontiers up to this size get kSmallRounds local rounds
constexpr int kSmallRounds = 16;
constexpr int kJobSeconds = 60;   // device-side limit of one decomposition job
constexpr uint32_t kPassChunk = kSweepThreads;   // smallest chunk of a node pass (SELECT, ASSIGN, ...)
constexpr uint32_t kBatchGrowChunk = kSweepThreads;        // jobs of several graphs: smallest growth chunk
constexpr uint32_t kBatchPassChunk = 16 * kSweepThreads;   // ... and smallest node-pass chunk (items)
constexpr uint32_t kRmaxSlots = 1024;   // RMAX: LDS table of cluster maxima (direct-mapped by center id)
constexpr uint32_t kRmaxFree = 0xffffffffu;
static_assert(kRmaxSlots == 1024, "RMAX slots are the top 10 bits of a 32-bit hash");
constexpr uint32_t kPullArcs = 8;   // pull-mode switch: heavy blocked arcs per unreached node
constexpr int64_t kHubDegree = 8;   // hub rows: more than kHubDegree x the average degree ...
constexpr int64_t kHubShare = 8;    // ... holding more than 1/kHubShare of the arcs: pull from the first stage

// ------------------------------------------------------------- control --

// Which counter holds the items of a phase's sweep, 3 bits per phase.  A
// table and two selects rather than a switch: the switch form (cases sharing
// a counter) compiled, for one phase, into divergent branches that never set
// the counter's address.
enum : uint32_t { IT_NONE = 0, IT_U = 1, IT_FCUR = 2, IT_BLK = 3, IT_FNXT = 4 };
constexpr uint64_t item_kind(uint32_t phase, uint32_t kind) { return (uint64_t)kind << (3 * phase); }
constexpr uint64_t kItemTable =
    item_kind(PH_SELECT, IT_U) | item_kind(PH_COMPACT, IT_U) | item_kind(PH_SINGLE, IT_U) |
    item_kind(PH_ASSIGN, IT_U) | item_kind(PH_RMAX, IT_U) | item_kind(PH_RELAX, IT_FCUR) |
    item_kind(PH_NEXT, IT_BLK) | item_kind(PH_MERGE, IT_BLK) | item_kind(PH_COMMIT, IT_FNXT) |
    item_kind(PH_C2_SELECT, IT_U) | item_kind(PH_C2_ASSIGN, IT_U) | item_kind(PH_C2_BOUNDARY, IT_BLK) |
    item_kind(PH_PULL, IT_U) | item_kind(PH_NEXT_PULL, IT_U);
static_assert(3 * PH_NEXT_PULL + 3 <= 64, "item table holds every phase");

__device__ uint32_t items_of(const GState &s, const GCount &c) {
  const uint32_t p = s.phase;
  const uint32_t kind = p <= PH_NEXT_PULL ? (uint32_t)(kItemTable >> (3 * p)) & 7u : IT_NONE;
  if (kind == IT_NONE) return 0;
  const uint32_t idx = kind == IT_FCUR ? s.fcur : (kind == IT_BLK ? s.blk : (kind == IT_FNXT ? s.fnxt : s.ucur));
  const PadU32 *list = kind == IT_U ? c.cntU : c.cnt;
  return list[idx].v;
}

// A failing graph stops alone; the other graphs of the job go on.
__device__ void fail(GState &s, Ctl *ctl, int status) {
  (void)ctl;
  s.status = status;
  s.phase = PH_DONE;
}

__device__ void begin_stage(const GDesc &d, GState &s, GCount &c, Ctl *ctl) {
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
  c.centers.v = 0;
  c.cntC.v = 0;
  s.phase = PH_SELECT;
}

// Upper end (exclusive) of the distance bucket that starts at lo.
__device__ __forceinline__ uint32_t bucket_limit(const GDesc &d, uint32_t lo) {
  if (d.bucket == 0) return 0xffffffffu;
  const uint64_t t = (uint64_t)lo + d.bucket;
  return t < 0xffffffffull ? (uint32_t)t : 0xffffffffu;
}

// Upper end (exclusive) of the narrower bucket of rows of more than mid_deg
// arcs.  Relaxing such a row before its node's distance is nearly final
// costs a full rescan when the distance drops again, so these rows wait
// until the frontier minimum comes within Delta / 2^row_shift of them.
__device__ __forceinline__ uint32_t row_limit(const GDesc &d, uint32_t delta, uint32_t lo) {
  if (d.row_shift < 0 || lo == 0xffffffffu) return 0xffffffffu;
  const uint32_t w = delta >> d.row_shift;
  const uint64_t t = (uint64_t)lo + (w ? w : 1u);
  return t < 0xffffffffull ? (uint32_t)t : 0xffffffffu;
}

// CLUSTER2: iteration s.stage + 1 draws centers with probability 2^i / n.
__device__ void c2_begin_iteration(const GDesc &d, GState &s, GCount &c) {
  const int i = (int)s.stage + 1;
  const double p = ldexp(1.0, i) / (double)d.n;
  s.T = p >= 1.0 ? ((uint64_t)1 << 32) : (uint64_t)floor(p * 4294967296.0);
  c.centers.v = 0;
  c.cntC.v = 0;
  s.phase = PH_C2_SELECT;
}

// Synchronous steps: a new PartialGrowth call at the current Delta.
__device__ __forceinline__ void begin_call(GState &s, uint32_t sweep_id) {
  s.levels++;
  s.level_id = sweep_id;
  s.steps_call = 0;
  s.theta = 0xffffffffu;
  s.row_base = 0xffffffffu;
  s.phase = PH_RELAX;
}

// Synchronous steps: add the blocked list to the active list, then `after`.
__device__ __forceinline__ void merge_then(GState &s, uint32_t after) {
  s.after = after;
  s.phase = PH_MERGE;
}

// Pull mode pays once the heavy arcs of the blocked rows, which a push rescan
// and a push NEXT read, outweigh kPullArcs arcs per unreached node (about
// what pulling reads per node: its rows are sorted by weight and it stops at
// its first reached neighbour).
__device__ __forceinline__ bool pull_pays(const GCount &c, uint32_t unreached) {
  return c.blk_arcs.v > (unsigned long long)kPullArcs * unreached;
}

__device__ __forceinline__ bool double_delta(GState &s, Ctl *ctl) {
  if (2ull * s.delta > CLD_DELTA_MAX) {
    fail(s, ctl, CLDIAM_EOVERFLOW);
    return false;
  }
  s.delta *= 2;
  return true;
}

// Per-graph transition after a sweep of its current phase.
__device__ void control_graph(const Job &job, int g, uint32_t sweep_id) {
  const GDesc &d = job.desc[g];
  GState &s = job.st[g];
  GCount &c = job.cn[g];
  switch (s.phase) {
    case PH_START:
      s.delta = d.delta0;
      s.stage = 0;
      s.nU = (uint32_t)d.n;
      c.cntU[0].v = (uint32_t)d.n;
      s.ucur = 0;
      s.fcur = 0; s.fnxt = 1; s.blk = 2;
      c.cnt[0].v = c.cnt[1].v = c.cnt[2].v = 0;
      c.blk_arcs.v = 0;
      c.hub_arcs.v = 0;
      c.radius.v = 0;
      if ((uint64_t)s.delta > CLD_DELTA_MAX) { fail(s, job.ctl, CLDIAM_EOVERFLOW); break; }
      s.pull = d.pull_mode == CLDIAM_PULL_ALWAYS ? 1u : 0u;
      begin_stage(d, s, c, job.ctl);
      break;
    case PH_SELECT:
      // frontier = sources from the previous stage + the new centers, all at
      // distance 0
      s.centers_total += c.centers.v;
      if (d.variant == CLDIAM_VARIANT_STEPS) {
        // the outer loop's test comes first: enough new centers end the stage
        if (2ull * c.cntC.v >= (uint64_t)s.nU) { s.phase = PH_ASSIGN; break; }
        begin_call(s, sweep_id);
        break;
      }
      s.levels++;
      // a skewed degree distribution (hub rows holding a large share of the
      // arcs) goes with a low diameter: the growth then reaches most nodes
      // within a few hops, which a pull pass does for less than pushing
      if (!s.pull && s.stage == 0 && d.pull_mode == CLDIAM_PULL_AUTO && c.hub_arcs.v > d.hub_min) s.pull = 1;
      if (s.pull) {
        // the uncovered nodes pull from the assigned nodes and the new centers
        s.pull_base = 0;
        s.phase = PH_PULL;
        break;
      }
      s.level_id = sweep_id;
      s.theta = bucket_limit(d, 0);
      s.row_base = 0;
      c.fmin.v = 0xffffffffu;
      s.phase = PH_RELAX;
      break;
    case PH_PULL:
      // the pulled nodes are the frontier of the level
      s.level_id = sweep_id;
      s.theta = bucket_limit(d, s.pull_base);
      s.row_base = s.pull_base;
      c.fmin.v = 0xffffffffu;
      s.phase = PH_RELAX;
      break;
    case PH_RELAX:
      s.sweeps++;
      if (d.variant == CLDIAM_VARIANT_STEPS) {
        s.rounds++;
        s.steps_call++;
        s.fid = sweep_id - 1;   // the stamp of the step's updated nodes
        s.phase = PH_COMMIT;
        break;
      }
      if (c.cnt[s.fnxt].v > 0) {
        uint32_t t = s.fcur; s.fcur = s.fnxt; s.fnxt = t;
        c.cnt[s.fnxt].v = 0;
        // the next bucket starts at the smallest distance on the frontier
        const uint32_t th = c.fmin.v == 0xffffffffu ? 0xffffffffu : bucket_limit(d, c.fmin.v);
        if (th > s.theta) s.theta = th;
        if (c.fmin.v > s.row_base) s.row_base = c.fmin.v;
        c.fmin.v = 0xffffffffu;
      } else {
        c.cnt[s.fcur].v = 0;
        if (s.c2) s.phase = PH_C2_ASSIGN;
        else if (2ull * c.cntC.v >= (uint64_t)s.nU) s.phase = PH_ASSIGN;
        else {
          // pull from the unreached side once the heavy arcs of the blocked
          // rows (what a push rescan reads) outweigh the unreached nodes
          if (!s.pull && d.pull_mode == CLDIAM_PULL_AUTO && pull_pays(c, s.nU - c.cntC.v)) s.pull = 1;
          c.next.v = CLD_INF64;
          s.phase = s.pull ? PH_NEXT_PULL : PH_NEXT;
        }
      }
      break;
    case PH_COMMIT: {
      const uint32_t nn = c.cnt[s.fnxt].v;
      s.updates += nn;
      uint32_t t = s.fcur; s.fcur = s.fnxt; s.fnxt = t;   // the updated nodes are the next active set
      c.cnt[s.fnxt].v = 0;
      if (nn > 0 && 2ull * c.cntC.v >= (uint64_t)s.nU) {
        merge_then(s, PH_ASSIGN);
      } else if (nn > 0 && d.step_cap && s.steps_call >= d.step_cap) {
        if (!double_delta(s, job.ctl)) break;
        merge_then(s, PH_RELAX);
      } else if (nn > 0) {
        s.phase = PH_RELAX;
      } else {
        c.next.v = CLD_INF64;   // fixpoint: is any uncovered node reachable?
        s.phase = PH_NEXT;
      }
      break;
    }
    case PH_MERGE:
      c.cnt[s.blk].v = 0;
      if (s.after == PH_RELAX) begin_call(s, sweep_id);
      else s.phase = s.after;
      break;
    case PH_NEXT:
      if (d.variant == CLDIAM_VARIANT_STEPS) {
        if (c.next.v == CLD_INF64) {
          merge_then(s, PH_ASSIGN);
        } else if (double_delta(s, job.ctl)) {
          merge_then(s, PH_RELAX);
        }
        break;
      }
      if (c.next.v == CLD_INF64) {
        s.phase = PH_ASSIGN;
      } else {
        uint64_t dl = s.delta;
        do {
          if (2 * dl > CLD_DELTA_MAX) { fail(s, job.ctl, CLDIAM_EOVERFLOW); return; }
          dl *= 2;
          s.levels++;
        } while (dl < c.next.v);
        s.delta = (uint32_t)dl;
        // rescan the blocked nodes at the new Delta; fresh blocked list
        uint32_t t = s.fcur; s.fcur = s.blk; s.blk = t;
        c.cnt[s.blk].v = 0;
        c.blk_arcs.v = 0;
        s.level_id = sweep_id;
        s.theta = bucket_limit(d, (uint32_t)c.next.v);
        s.row_base = (uint32_t)c.next.v;
        c.fmin.v = 0xffffffffu;
        s.phase = PH_RELAX;
      }
      break;
    case PH_NEXT_PULL:
      if (c.next.v == CLD_INF64) {
        s.phase = PH_ASSIGN;
      } else {
        uint64_t dl = s.delta;
        do {
          if (2 * dl > CLD_DELTA_MAX) { fail(s, job.ctl, CLDIAM_EOVERFLOW); return; }
          dl *= 2;
          s.levels++;
        } while (dl < c.next.v);
        s.delta = (uint32_t)dl;
        c.cnt[s.blk].v = 0;
        c.blk_arcs.v = 0;
        s.pull_base = (uint32_t)c.next.v;
        s.phase = PH_PULL;
      }
      break;
    case PH_ASSIGN:
      s.phase = PH_RMAX;
      break;
    case PH_RMAX:
      c.cntU[s.ucur ^ 1].v = 0;
      s.phase = PH_COMPACT;
      break;
    case PH_COMPACT: {
      if (s.stage < CLDIAM_STAGE_LOG) {
        int32_t *lg = job.log + ((size_t)g * CLDIAM_STAGE_LOG + s.stage) * 4;
        lg[0] = (int32_t)s.nU; lg[1] = (int32_t)c.centers.v; lg[2] = (int32_t)c.cntC.v; lg[3] = (int32_t)s.delta;
      }
      s.ucur ^= 1;
      s.nU = c.cntU[s.ucur].v;
      s.stage++;
      if (s.c2) {
        // the blocked list stays: next iteration's Contract2 boundary
        c.cnt[s.fcur].v = 0;
        c.cnt[s.fnxt].v = 0;
        if (s.stage >= d.c2_iters) s.phase = PH_DONE;
        else c2_begin_iteration(d, s, c);
        break;
      }
      if (d.variant != CLDIAM_VARIANT_STEPS) {
        // sources of the next stage: the blocked list of the last level, or,
        // when it outnumbers the remaining uncovered nodes, none: those
        // nodes pull from their assigned neighbours instead
        if (!s.pull && d.pull_mode == CLDIAM_PULL_AUTO && pull_pays(c, c.cntU[s.ucur].v)) s.pull = 1;
        if (!s.pull) { uint32_t t = s.fcur; s.fcur = s.blk; s.blk = t; }
        else c.cnt[s.fcur].v = 0;
      }
      // (synchronous steps: the active list, merged with the blocked list,
      // already holds them)
      c.cnt[s.blk].v = 0;
      c.blk_arcs.v = 0;
      c.cnt[s.fnxt].v = 0;
      begin_stage(d, s, c, job.ctl);
      break;
    }
    case PH_SINGLE:
      s.singletons = s.nU;
      s.phase = PH_DONE;
      if (d.variant == CLDIAM_VARIANT_CLUSTER2) {
        // CLUSTER2 on top of the finished CLUSTER run
        const uint64_t r1 = c.radius.v;
        if (2 * r1 > CLD_DELTA_MAX) { fail(s, job.ctl, CLDIAM_EOVERFLOW); break; }
        s.radius1 = r1;
        s.delta = (uint32_t)(2 * r1);
        if (d.c2_iters == 0) break;   // one node: its own cluster
        s.c2 = 1;
        s.pull = 0;
        s.stage = 0;
        s.levels = 0;
        s.centers_total = 0;
        s.singletons = 0;
        c.radius.v = 0;
        s.phase = PH_C2_INIT;
      }
      break;
    case PH_C2_INIT:
      s.nU = (uint32_t)d.n;
      s.ucur = 0;
      c.cntU[0].v = (uint32_t)d.n;
      c.cnt[0].v = c.cnt[1].v = c.cnt[2].v = 0;
      c2_begin_iteration(d, s, c);
      break;
    case PH_C2_SELECT:
      s.centers_total += c.centers.v;
      s.levels++;
      s.phase = PH_C2_BOUNDARY;
      break;
    case PH_C2_BOUNDARY:
      // the boundary list is consumed; growth marks a fresh one
      c.cnt[s.blk].v = 0;
      s.level_id = sweep_id;
      s.theta = bucket_limit(d, 0);
      s.row_base = 0;
      c.fmin.v = 0xffffffffu;
      s.phase = PH_RELAX;
      break;
    case PH_C2_ASSIGN:
      c.cntU[s.ucur ^ 1].v = 0;
      s.phase = PH_COMPACT;
      break;
    default:
      break;
  }
}

// One workgroup of T threads: control of every graph, then the next sweep's
// index space.
template <int T>
__device__ void control_block(const Job &job) {
  __shared__ uint32_t scan[T];
  __shared__ uint32_t carry, alldone;
  __shared__ unsigned long long work;
  Ctl *ctl = job.ctl;
  uint32_t sweep_id = ctl->sweep_id + 1;
  if (threadIdx.x == 0) {
    carry = 0;
    alldone = 1;
    work = 0;
    const unsigned long long now = wall_clock64();
    if (ctl->iterations == 0) ctl->t_start = now;
    else if (now - ctl->t_start > ctl->t_limit && ctl->error == 0) atomicCAS(&ctl->error, 0u, (uint32_t)(-CLDIAM_ETIMEOUT));
  }
  __syncthreads();
  // every graph's transition and the items of its next sweep
  for (int base = 0; base < job.G; base += T) {
    const int g = base + (int)threadIdx.x;
    if (g < job.G) {
      if (ctl->error == 0 || job.st[g].phase == PH_DONE) control_graph(job, g, sweep_id);
      if (ctl->error != 0 && job.st[g].phase != PH_DONE) job.st[g].phase = PH_DONE;
      const uint32_t phase = job.st[g].phase;
      const uint32_t n_items =
          job.st[g].phase == PH_C2_INIT ? (uint32_t)job.desc[g].n : items_of(job.st[g], job.cn[g]);
      job.seg[2 * job.G + 1 + g] = n_items;
      if (n_items) atomicAdd(&work, (unsigned long long)n_items);
      if (phase != PH_DONE && phase != PH_IDLE) atomicAnd(&alldone, 0u);
    }
  }
  __syncthreads();
  // In a job of several graphs no chunk is smaller than the sweep's average
  // items per workgroup (up to kBatchGrowChunk / kBatchPassChunk): a small
  // frontier or node list then takes a few larger chunks instead of one per
  // workgroup, each of which would pay a chunk's fixed cost (setup,
  // barriers, local rounds) for a handful of items.
  const unsigned long long avg = work / (unsigned long long)job.nblocks;
  for (int base = 0; base < job.G; base += T) {
    const int g = base + (int)threadIdx.x;
    uint32_t items = 0;
    if (g < job.G) {
      const uint32_t phase = job.st[g].phase;
      const uint32_t n_items = job.seg[2 * job.G + 1 + g];
      // Otherwise every graph is cut into its own chunks, at most chunk_factor
      // per workgroup, so that the frontier of each graph is spread over the
      // whole grid whatever the other graphs of the job are doing (a node pass
      // of millions of cheap items beside a small frontier of costly rows).
      uint32_t per = 0;
      if (n_items) {
        const bool grow = phase == PH_RELAX || phase == PH_NEXT || phase == PH_PULL || phase == PH_NEXT_PULL;
        const uint32_t nch = (uint32_t)job.nblocks * (grow ? (uint32_t)job.desc[g].chunk_factor : 1u);
        per = (n_items + nch - 1) / nch;
        if (!grow && per < kPassChunk) per = kPassChunk;
        if (job.G > 1) {
          const unsigned long long cap = grow ? kBatchGrowChunk : kBatchPassChunk;
          const uint32_t least = (uint32_t)(avg < cap ? avg : cap);
          if (per < least) per = least;
        }
        items = (n_items + per - 1) / per;
      }
      job.seg[job.G + 1 + g] = per;
    }
    scan[threadIdx.x] = items;
    __syncthreads();
    for (int o = 1; o < T; o <<= 1) {
      uint32_t x = threadIdx.x >= (unsigned)o ? scan[threadIdx.x - o] : 0;
      __syncthreads();
      scan[threadIdx.x] += x;
      __syncthreads();
    }
    if (g < job.G) job.seg[g] = carry + scan[threadIdx.x] - items;
    __syncthreads();
    if (threadIdx.x == T - 1) carry += scan[T - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    job.seg[job.G] = carry;
    ctl->total = carry;
    ctl->cursor.v = 0;
    ctl->idle.v = 0;
    ctl->sweep_id = sweep_id;
    ctl->iterations++;
    ctl->done = alldone;
    if (job.hmirror) {
      __hip_atomic_store(&job.hmirror[0], ctl->iterations, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&job.hmirror[1], alldone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  __syncthreads();
}

// --------------------------------------------------------------- sweeps --

struct Out {
  int32_t *list;     // list base for this graph (offset applied)
  uint32_t *count;   // its global counter
};

// LDS staging of up to three output lists of one graph run.
struct Stage {
  int32_t buf[3][kStageCap];
  union {
    int32_t lq[2][kLocalCap];  // RELAX: local relaxation queues
    struct {                   // RMAX: per-cluster maxima of this workgroup's nodes
      uint32_t tag[kRmaxSlots];
      unsigned long long mx[kRmaxSlots];
    } rmax;
  };
  uint32_t lq_cnt[2];
  int32_t mid[kMidCap];      // rows deferred to one wave each
  int32_t big[kBigCap];      // rows deferred to the whole workgroup
  uint32_t mid_cnt, big_cnt;
  unsigned long long blk_min;  // workgroup minimum for the NEXT scan of a big row
  unsigned long long row_key;  // key of the big row being scanned
  int32_t row_lo;              // end of its light prefix (index within the row)
  int32_t row_start;           // first arc of its scan (index within the row)
  uint32_t blk_hit;
  uint32_t cnt[3];
  uint32_t base[3];
  unsigned long long acc;   // min (NEXT) or max (ASSIGN) accumulator
  unsigned long long blk_arcs;   // RELAX: heavy arcs of the rows this workgroup put on the blocked list
  uint32_t acc32;           // centers drawn (SELECT)
  uint32_t flush;           // a list passed the flush threshold
  uint32_t fmin;            // RELAX: smallest distance pushed on the next frontier
  uint32_t chunk;           // next chunk of this workgroup
  uint32_t stop;            // local rounds end early: most of the grid has finished the sweep
  Out out[3];               // output lists of the current run (in LDS: the flush indexes them by list number)
};

// Stage v on output list k; falls back to a direct global slot when the LDS
// buffer is full (only possible for rows with thousands of improved arcs).
__device__ __forceinline__ void stage_push(Stage &S, const Out *out, int k, int32_t v) {
  const uint32_t slot = atomicAdd(&S.cnt[k], 1u);
  if (slot < kStageCap) {
    S.buf[k][slot] = v;
  } else {
    out[k].list[atomicAdd(out[k].count, 1u)] = v;
  }
}

// Writes the staged entries out: one global reservation per list.
__device__ void stage_flush(Stage &S, const Out *out, int nout) {
  __syncthreads();
  if (threadIdx.x < (unsigned)nout) {
    const int k = threadIdx.x;
    const uint32_t n = S.cnt[k] < kStageCap ? S.cnt[k] : kStageCap;
    uint32_t *count = k == 0 ? out[0].count : (k == 1 ? out[1].count : out[2].count);
    S.base[k] = n ? atomicAdd(count, n) : 0;
    S.cnt[k] = n;
  }
  __syncthreads();
  {
    const uint32_t n = S.cnt[0], b = S.base[0];
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) out[0].list[b + i] = S.buf[0][i];
  }
  if (nout > 1) {
    const uint32_t n = S.cnt[1], b = S.base[1];
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) out[1].list[b + i] = S.buf[1][i];
  }
  if (nout > 2) {
    const uint32_t n = S.cnt[2], b = S.base[2];
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) out[2].list[b + i] = S.buf[2][i];
  }
  __syncthreads();
  if (threadIdx.x < 3) S.cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) S.flush = 0;
  __syncthreads();
}

// Synchronous step for one active node u (see relax_one_sync).  Returns the
// number of offers sent (arcs with d_u + w <= Delta).
__device__ __forceinline__ uint32_t relax_sync(const Job &job, const GDesc &d, int64_t off, uint32_t delta,
                                               uint32_t it, uint32_t level_id, int32_t u, Stage &S,
                                               const Out *out);

// Smallest tentative distance pushed on the next frontier by this workgroup.
__device__ __forceinline__ void note_fmin(Stage &S, uint32_t dist) {
  if (dist < S.fmin) atomicMin(&S.fmin, dist);
}

// RELAX: scan the light prefix of u's row (w <= Delta - d_u) and offer
// (d_u + w, c_u) to every neighbour.  Outputs: 0 next frontier, 1 covered,
// 2 blocked.  Arcs are handled four at a time so that their key loads and
// atomics are in flight together.  Improved neighbours are also appended to
// the workgroup's local queue `lq` (when it has room) for the local rounds.
constexpr int kArcBatch = 4;

// Queues a long row for the cooperative passes of this round; false when the
// queue is full (the caller then handles the row itself).
__device__ __forceinline__ bool defer_row(Stage &S, int32_t u, int32_t deg, int32_t big_deg) {
  if (deg > big_deg) {
    const uint32_t slot = atomicAdd(&S.big_cnt, 1u);
    if (slot < kBigCap) { S.big[slot] = u; return true; }
  } else {
    const uint32_t slot = atomicAdd(&S.mid_cnt, 1u);
    if (slot < kMidCap) { S.mid[slot] = u; return true; }
  }
  return false;
}

__device__ __forceinline__ void lq_push(uint32_t *lq_cnt, int32_t *lq, int32_t v, uint32_t cap) {
  const uint32_t slot = atomicAdd(lq_cnt, 1u);
  if (slot < cap) lq[slot] = v;
}

__device__ __forceinline__ uint32_t relax_item(const Job &job, const GDesc &d, int64_t off, uint32_t delta,
                                               uint32_t theta, uint32_t theta_row, uint32_t it,
                                               uint32_t level_id, int32_t u,
                                               Stage &S, const Out *out, uint32_t *lq_cnt, int32_t *lq) {
  const uint64_t ku = job.key[off + u];
  int64_t a0 = 0;
  int32_t deg = 0;   // a row has fewer than 2^31 arcs: indices within it are 32-bit
  bool later = (uint32_t)(ku >> 32) >= theta;
  if (!later) {
    a0 = d.row_ptr[u];
    deg = (int32_t)(d.row_ptr[u + 1] - a0);
    later = deg > d.mid_deg && (uint32_t)(ku >> 32) >= theta_row;
  }
  if (later) {
    // beyond the current distance bucket: stays on the frontier for a later
    // sweep (it may already be there if it improved in this sweep)
    if (atomicExch(&job.fstamp[off + u], it) != it) {
      stage_push(S, out, 0, u);
      note_fmin(S, (uint32_t)(ku >> 32));
    }
    return 0;
  }
  if (deg > d.mid_deg && defer_row(S, u, deg, d.big_deg)) return 0;
  const uint64_t *row = d.arcs + a0;
  const uint32_t lim = delta - (uint32_t)(ku >> 32);
  bool blocked = false;
  uint32_t scanned = 0;
  for (int32_t base = 0; base < deg && !blocked; base += kArcBatch) {
    uint64_t arc[kArcBatch], cur[kArcBatch];
    bool ok[kArcBatch];
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) arc[j] = base + j < deg ? row[base + j] : ~0ull;
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) {
      const bool in = base + j < deg;
      ok[j] = in && (uint32_t)(arc[j] >> 32) <= lim;
      if (in && !ok[j]) blocked = true;
      scanned += ok[j];
    }
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) cur[j] = ok[j] ? job.key[off + (int32_t)(uint32_t)arc[j]] : 0ull;
    // An offer that beats the key it read is applied with atomicMin and, in
    // the same round trip, stamps the target for the next frontier.  The
    // stamp may be taken by an offer that then loses to a concurrent better
    // one; the node is then still on the frontier (harmless), and an improver
    // never finds the node missing from it.  The returned stamp also keeps each
    // node to one entry per list and sweep, which the lists' capacity (n) needs.
    bool front[kArcBatch];
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) {
      const uint64_t cand = ku + (arc[j] & 0xffffffff00000000ull);
      ok[j] = ok[j] && cand < cur[j];
      const int64_t gv = off + (int32_t)(uint32_t)arc[j];
      cur[j] = ok[j] ? atomicMin((unsigned long long *)&job.key[gv], (unsigned long long)cand) : 0ull;
      front[j] = ok[j] && atomicExch(&job.fstamp[gv], it) != it;
      ok[j] = ok[j] && cand < cur[j];
    }
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) {
      const int32_t v = (int32_t)(uint32_t)arc[j];
      if (front[j]) {
        stage_push(S, out, 0, v);
        note_fmin(S, (uint32_t)(ku >> 32) + (uint32_t)(arc[j] >> 32));
      }
      if (!ok[j]) continue;
      if (cur[j] == CLD_INF64) stage_push(S, out, 1, v);
      if (lq) lq_push(lq_cnt, lq, v, d.lq_cap);
    }
  }
  if (blocked && job.bstamp[off + u] != level_id && atomicExch(&job.bstamp[off + u], level_id) != level_id) {
    stage_push(S, out, 2, u);
    atomicAdd(&S.blk_arcs, (unsigned long long)(deg - (int32_t)scanned));   // the light arcs come first
  }
  return scanned;
}

__device__ __forceinline__ uint32_t relax_sync(const Job &job, const GDesc &d, int64_t off, uint32_t delta,
                                               uint32_t it, uint32_t level_id, int32_t u, Stage &S,
                                               const Out *out) {
  const int64_t a0 = d.row_ptr[u];
  const int32_t deg = (int32_t)(d.row_ptr[u + 1] - a0);
  if (deg > d.mid_deg && defer_row(S, u, deg, d.big_deg)) return 0;
  const uint64_t *row = d.arcs + a0;
  const uint64_t ku = job.key[off + u];
  const uint32_t lim = delta - (uint32_t)(ku >> 32);
  bool blocked = false;
  uint32_t scanned = 0;
  for (int32_t base = 0; base < deg && !blocked; base += kArcBatch) {
    uint64_t arc[kArcBatch], cur[kArcBatch], old[kArcBatch];
    bool ok[kArcBatch], front[kArcBatch];
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) arc[j] = base + j < deg ? row[base + j] : ~0ull;
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) {
      const bool in = base + j < deg;
      ok[j] = in && (uint32_t)(arc[j] >> 32) <= lim;
      if (in && !ok[j]) blocked = true;
      scanned += ok[j];
    }
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) cur[j] = ok[j] ? job.key[off + (int32_t)(uint32_t)arc[j]] : 0ull;
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) {
      const uint64_t cand = ku + (arc[j] & 0xffffffff00000000ull);
      ok[j] = ok[j] && (cand >> 32) < (cur[j] >> 32);
      const int64_t gv = off + (int32_t)(uint32_t)arc[j];
      old[j] = ok[j] ? atomicMin((unsigned long long *)&job.keyn[gv], (unsigned long long)cand) : 0ull;
      front[j] = ok[j] && atomicExch(&job.fstamp[gv], it) != it;
    }
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) {
      const int32_t v = (int32_t)(uint32_t)arc[j];
      if (front[j]) stage_push(S, out, 0, v);
      if (ok[j] && old[j] == CLD_INF64) stage_push(S, out, 1, v);
    }
  }
  if (blocked && job.bstamp[off + u] != level_id && atomicExch(&job.bstamp[off + u], level_id) != level_id)
    stage_push(S, out, 2, u);
  return scanned;
}

// One arc of a cooperative row: the same offer as in relax_item.
__device__ __forceinline__ void relax_one(const Job &job, int64_t off, uint64_t ku, uint64_t arc, uint32_t it,
                                          Stage &S, const Out *out, uint32_t *lq_cnt, int32_t *lq, uint32_t lq_cap) {
  const int32_t v = (int32_t)(uint32_t)arc;
  const int64_t gv = off + v;
  const uint64_t cand = ku + (arc & 0xffffffff00000000ull);
  if (cand < job.key[gv]) {
    const uint64_t old = atomicMin((unsigned long long *)&job.key[gv], (unsigned long long)cand);
    if (atomicExch(&job.fstamp[gv], it) != it) {
      stage_push(S, out, 0, v);
      note_fmin(S, (uint32_t)(cand >> 32));
    }
    if (cand < old) {
      if (old == CLD_INF64) stage_push(S, out, 1, v);
      if (lq) lq_push(lq_cnt, lq, v, lq_cap);
    }
  }
}

// Synchronous steps: an offer is judged against the state before the step
// (key) and applied to the state after it (keyn); only a strictly smaller
// distance is accepted, the lexicographic minimum over the step's offers wins.
__device__ __forceinline__ void relax_one_sync(const Job &job, int64_t off, uint64_t ku, uint64_t arc, uint32_t it,
                                               Stage &S, const Out *out) {
  const int32_t v = (int32_t)(uint32_t)arc;
  const int64_t gv = off + v;
  const uint64_t cand = ku + (arc & 0xffffffff00000000ull);
  if ((cand >> 32) < (job.key[gv] >> 32)) {
    const uint64_t old = atomicMin((unsigned long long *)&job.keyn[gv], (unsigned long long)cand);
    if (atomicExch(&job.fstamp[gv], it) != it) stage_push(S, out, 0, v);
    if (old == CLD_INF64) stage_push(S, out, 1, v);
  }
}

__device__ __forceinline__ void mark_blocked(const Job &job, int64_t off, int32_t u, uint32_t level_id, int32_t heavy,
                                             Stage &S, const Out *out) {
  if (job.bstamp[off + u] != level_id && atomicExch(&job.bstamp[off + u], level_id) != level_id) {
    stage_push(S, out, 2, u);
    atomicAdd(&S.blk_arcs, (unsigned long long)heavy);
  }
}

// NEXT for a short row: smallest d_u + w over its heavy arcs (w > Delta - d_u)
// into unreached nodes.  Rows are sorted by weight, so the first such arc in
// ascending order gives the minimum.
__device__ __forceinline__ uint64_t next_small(const Job &job, const GDesc &d, int64_t off, uint32_t delta,
                                               int32_t u) {
  const uint64_t ku = job.key[off + u];
  const uint32_t du = (uint32_t)(ku >> 32);
  const uint32_t lim = delta - du;
  const int64_t a0 = d.row_ptr[u];
  const uint64_t *row = d.arcs + a0;
  const int32_t deg = (int32_t)(d.row_ptr[u + 1] - a0);
  for (int32_t a = 0; a < deg; ++a) {
    const uint64_t arc = row[a];
    const uint32_t w = (uint32_t)(arc >> 32);
    if (w <= lim) continue;
    if (job.key[off + (int32_t)(uint32_t)arc] == CLD_INF64) return (uint64_t)du + w;
  }
  return CLD_INF64;
}

// Long rows remember their last scan (key and light limit).  Within a Delta
// level a node's key only decreases and Delta is fixed, so a record with the
// node's current key means that every arc up to the recorded limit has
// already been offered with this key; once a level is at its fixpoint the
// reached nodes' keys are final, so a larger Delta only has to look past the
// recorded limit; and after a stage the arcs up to it lead to assigned nodes.
// A record read in a race is never larger than what some scan with an equal
// or better key has covered, so skipping up to it drops no useful offer.
// First arc in [lo, hi) of a weight-sorted row with w > x, found by the 64
// lanes of a wave together: each round samples 64 evenly spaced arcs and
// keeps the bracket of the first one above x (two or three dependent loads
// for rows up to 8192 arcs instead of a dozen for a binary search).  Every
// lane of the wave calls it with the same arguments and gets the result.
__device__ __forceinline__ int32_t wave_first_above(const uint64_t *arcs, int32_t lo, int32_t hi, uint32_t x) {
  const int32_t lane = (int32_t)(threadIdx.x & 63);
  while (hi - lo > 64) {
    const int32_t step = (hi - lo + 63) >> 6;
    const int32_t p = lo + lane * step;
    const bool above = p < hi && (uint32_t)(arcs[p] >> 32) > x;
    const unsigned long long m = __ballot(above);
    if (m == 0) {
      // every valid sample is <= x: the answer lies after the last one
      const int32_t last = lo + ((hi - 1 - lo) / step) * step;
      lo = last + 1;
    } else {
      const int32_t f = __ffsll((long long)m) - 1;
      const int32_t nlo = f == 0 ? lo : lo + (f - 1) * step + 1;
      hi = lo + f * step;   // the sample at f is above x
      lo = nlo;
      if (f == 0) return hi;
    }
  }
  const int32_t p = lo + lane;
  const unsigned long long m = __ballot(p < hi && (uint32_t)(arcs[p] >> 32) > x);
  return m ? lo + (__ffsll((long long)m) - 1) : hi;
}

// Resume index within the row [0, end) of u (arcs at row).
__device__ __forceinline__ int32_t resume_at_wave(const Job &job, int64_t off, int32_t u, uint64_t ku,
                                                  const uint64_t *row, int32_t end) {
  if (job.keyn[off + u] != ku) return 0;
  return wave_first_above(row, 0, end, job.slim[off + u]);
}

__device__ __forceinline__ void note_scan(const Job &job, int64_t off, int32_t u, uint64_t ku, uint32_t lim) {
  job.slim[off + u] = lim;
  job.keyn[off + u] = ku;
}

// Cooperative passes over the rows deferred in this round: each wave takes
// whole mid-size rows (64 arcs per step), then the whole workgroup takes each
// big row (blockDim arcs per step).  mode 0 relaxes the light prefix; mode 2
// does the same as a synchronous step; mode 1 (NEXT) finds the first heavy arc
// into an unreached node and folds d_u + w into S.acc.
__device__ uint32_t coop_rows(const Job &job, const GDesc &d, int64_t off, uint32_t delta, uint32_t it,
                              uint32_t level_id, Stage &S, const Out *out, uint32_t *lq_cnt, int32_t *lq, int mode,
                              bool resume) {
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const uint32_t nm = S.mid_cnt < kMidCap ? S.mid_cnt : kMidCap;
  const uint32_t nb = S.big_cnt < kBigCap ? S.big_cnt : kBigCap;
  uint32_t scanned = 0;
  for (uint32_t r = wave; r < nm; r += nwaves) {
    const int32_t u = S.mid[r];
    const int64_t a0 = d.row_ptr[u];
    const int32_t a1 = (int32_t)(d.row_ptr[u + 1] - a0);   // row-relative from here on
    const uint64_t *row = d.arcs + a0;
    const uint64_t ku = job.key[off + u];
    const uint32_t lim = delta - (uint32_t)(ku >> 32);
    if (mode != 1) {
      const int32_t start = resume ? resume_at_wave(job, off, u, ku, row, a1) : 0;
      int32_t light_end = start;   // the light arcs are a prefix of the row
      for (int32_t base = start; base < a1; base += 64) {
        const int32_t a = base + (int32_t)lane;
        const uint64_t arc = a < a1 ? row[a] : ~0ull;
        const bool light = a < a1 && (uint32_t)(arc >> 32) <= lim;
        const int nl = __popcll(__ballot(light));
        light_end = base + nl;
        if (nl == 0) break;
        if (light) {
          ++scanned;
          if (mode == 2) relax_one_sync(job, off, ku, arc, it, S, out);
          else relax_one(job, off, ku, arc, it, S, out, lq_cnt, lq, d.lq_cap);
        }
        if (nl < 64) break;
      }
      if (lane == 0 && (uint32_t)(row[a1 - 1] >> 32) > lim)
        mark_blocked(job, off, u, level_id, a1 - light_end, S, out);
      if (resume && lane == 0) note_scan(job, off, u, ku, lim);
    } else {
      // the heavy arcs start after the light prefix
      for (int32_t base = wave_first_above(row, 0, a1, lim); base < a1; base += 64) {
        const int32_t a = base + (int32_t)lane;
        const uint64_t arc = a < a1 ? row[a] : 0ull;
        const uint32_t w = (uint32_t)(arc >> 32);
        const bool hit = a < a1 && w > lim && job.key[off + (int32_t)(uint32_t)arc] == CLD_INF64;
        const unsigned long long m = __ballot(hit);
        if (m) {
          // first hit in ascending order has the smallest weight
          const int src = __ffsll((long long)m) - 1;
          const uint64_t c = (uint64_t)(uint32_t)(ku >> 32) + (uint32_t)(__shfl(arc, src) >> 32);
          if (lane == 0 && c < S.acc) atomicMin(&S.acc, (unsigned long long)c);
          break;
        }
      }
    }
  }
  for (uint32_t h = 0; h < nb; ++h) {
    const int32_t u = S.big[h];
    const int64_t a0 = d.row_ptr[u];
    const int32_t a1 = (int32_t)(d.row_ptr[u + 1] - a0);   // row-relative from here on
    const uint64_t *row = d.arcs + a0;
    // wave 0 reads u's key once for the whole workgroup (so every thread scans
    // with the same key and the scan record describes all of them) and finds
    // the end of the light prefix and the resume point
    if (threadIdx.x < 64) {
      const uint64_t k = job.key[off + u];
      const int32_t light_end = wave_first_above(row, 0, a1, delta - (uint32_t)(k >> 32));
      const int32_t from = (mode != 1 && resume) ? resume_at_wave(job, off, u, k, row, light_end) : 0;
      if (threadIdx.x == 0) {
        S.row_key = k;
        S.row_lo = light_end;
        S.row_start = from;
      }
    }
    __syncthreads();
    const uint64_t ku = S.row_key;
    const uint32_t lim = delta - (uint32_t)(ku >> 32);
    const int32_t lo = S.row_lo;   // first index with w > lim
    if (mode != 1) {
      const int32_t start = S.row_start;
      for (int32_t a = start + (int32_t)threadIdx.x; a < lo; a += (int32_t)blockDim.x) {
        ++scanned;
        if (mode == 2) relax_one_sync(job, off, ku, row[a], it, S, out);
        else relax_one(job, off, ku, row[a], it, S, out, lq_cnt, lq, d.lq_cap);
      }
      if (threadIdx.x == 0 && lo < a1) mark_blocked(job, off, u, level_id, a1 - lo, S, out);
      // keep LDS staging within bounds between rows
      __syncthreads();
      // every thread's part of the row is done: record the scan
      if (resume && threadIdx.x == 0) note_scan(job, off, u, ku, lim);
      if (threadIdx.x < 3 && S.cnt[threadIdx.x] > kStageCap - kSweepThreads) S.flush = 1;
      __syncthreads();
      if (S.flush) stage_flush(S, out, 3);
    } else {
      for (int32_t base = lo; base < a1; base += (int32_t)blockDim.x) {
        if (threadIdx.x == 0) { S.blk_min = CLD_INF64; S.blk_hit = 0; }
        __syncthreads();
        const int32_t a = base + (int32_t)threadIdx.x;
        if (a < a1) {
          const uint64_t arc = row[a];
          if (job.key[off + (int32_t)(uint32_t)arc] == CLD_INF64) {
            const uint64_t c = (uint64_t)(uint32_t)(ku >> 32) + (uint32_t)(arc >> 32);
            atomicMin(&S.blk_min, (unsigned long long)c);
            S.blk_hit = 1;
          }
        }
        __syncthreads();
        const bool found = S.blk_hit != 0;
        if (found && threadIdx.x == 0 && S.blk_min < S.acc) atomicMin(&S.acc, S.blk_min);
        __syncthreads();
        if (found) break;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) { S.mid_cnt = 0; S.big_cnt = 0; }
  __syncthreads();
  return scanned;
}

// Pull mode.  Offers over arcs that were heavy at the previous Delta, or
// from the sources of a new stage, can only reach unreached nodes: they are
// at least the previous Delta, above every reached key.  When the unreached
// nodes are fewer than the blocked ones, they look at their neighbours
// instead: PULL gives an unreached node v the lexicographic minimum over its
// neighbours u with a key of (d_u + w, c_u), d_u + w <= Delta (only v's own
// thread writes v's key, so no atomic is needed); NEXT_PULL folds the smallest
// d_u + w over the same arcs into S.acc.  Rows are sorted by weight, so both
// stop early (pull_more).
// A key read while its node is being pulled in the same pass is a real path
// too, so taking it only moves the fixpoint closer.

// Whether an arc of weight w, in a row sorted by weight, can still beat the
// best offer: every offer over it is at least w (d_u >= 0), so PULL stops
// past min(Delta, best distance) (an equal distance may still win on the
// center id) and NEXT_PULL once w reaches the best distance.
__device__ __forceinline__ bool pull_more(uint64_t w, uint64_t best, uint32_t delta, bool next) {
  return next ? w < best : (w <= delta && w <= (best >> 32));
}

// Value of one arc (pull) or distance (next) offered to an unreached node.
__device__ __forceinline__ uint64_t pull_offer(const Job &job, int64_t off, uint64_t arc, uint32_t delta, bool next) {
  const uint64_t k = job.key[off + (int32_t)(uint32_t)arc];
  if (k == CLD_INF64) return CLD_INF64;
  const uint64_t du = k >> 32, w = arc >> 32;
  if (next) return du + w;
  return du + w <= delta ? k + (w << 32) : CLD_INF64;
}

__device__ __forceinline__ void pull_apply(const Job &job, int64_t off, int32_t v, uint64_t best, bool next, Stage &S,
                                           const Out *out) {
  if (next) {
    if (best < S.acc) atomicMin(&S.acc, (unsigned long long)best);
  } else if (best != CLD_INF64) {
    job.key[off + v] = best;
    stage_push(S, out, 0, v);
    stage_push(S, out, 1, v);
  }
}

// One node of the uncovered list, its row scanned by this thread (long rows
// are deferred to a wave or to the workgroup).
__device__ __forceinline__ void pull_item(const Job &job, const GDesc &d, int64_t off, uint32_t delta, int32_t v,
                                          bool next, Stage &S, const Out *out) {
  if (job.key[off + v] != CLD_INF64) return;
  const int64_t a0 = d.row_ptr[v];
  const int32_t deg = (int32_t)(d.row_ptr[v + 1] - a0);
  if (deg > d.mid_deg && defer_row(S, v, deg, d.big_deg)) return;
  const uint64_t *row = d.arcs + a0;
  uint64_t best = CLD_INF64;
  for (int32_t base = 0; base < deg; base += kArcBatch) {
    uint64_t arc[kArcBatch];
    bool ok[kArcBatch];
    bool stop = false;
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) arc[j] = base + j < deg ? row[base + j] : ~0ull;
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) {
      const uint64_t w = arc[j] >> 32;
      ok[j] = base + j < deg && pull_more(w, best, delta, next);
      if (base + j < deg && !ok[j]) stop = true;
    }
    uint64_t c[kArcBatch];
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) c[j] = ok[j] ? pull_offer(job, off, arc[j], delta, next) : CLD_INF64;
#pragma unroll
    for (int j = 0; j < kArcBatch; ++j) best = c[j] < best ? c[j] : best;
    if (stop) break;
  }
  pull_apply(job, off, v, best, next, S, out);
}

__device__ __forceinline__ uint64_t wave_min_all(uint64_t x) {
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t y = __shfl_xor(x, o);
    x = y < x ? y : x;
  }
  return x;
}

// The long rows deferred by pull_item: a wave per row, then the whole
// workgroup per hub row.
__device__ void pull_rows(const Job &job, const GDesc &d, int64_t off, uint32_t delta, bool next, Stage &S,
                          const Out *out) {
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const uint32_t nm = S.mid_cnt < kMidCap ? S.mid_cnt : kMidCap;
  const uint32_t nb = S.big_cnt < kBigCap ? S.big_cnt : kBigCap;
  for (uint32_t r = wave; r < nm; r += nwaves) {
    const int32_t v = S.mid[r];
    const int64_t a0 = d.row_ptr[v];
    const int32_t a1 = (int32_t)(d.row_ptr[v + 1] - a0);
    const uint64_t *row = d.arcs + a0;
    uint64_t best = CLD_INF64;
    for (int32_t base = 0; base < a1; base += 64) {
      const int32_t a = base + (int32_t)lane;
      const uint64_t arc = a < a1 ? row[a] : ~0ull;
      const uint64_t w = arc >> 32;
      const bool in = a < a1 && pull_more(w, best, delta, next);
      if (!__any(in)) break;
      const uint64_t m = wave_min_all(in ? pull_offer(job, off, arc, delta, next) : CLD_INF64);
      best = m < best ? m : best;
    }
    if (lane == 0) pull_apply(job, off, v, best, next, S, out);
  }
  for (uint32_t h = 0; h < nb; ++h) {
    const int32_t v = S.big[h];
    const int64_t a0 = d.row_ptr[v];
    const int32_t a1 = (int32_t)(d.row_ptr[v + 1] - a0);
    const uint64_t *row = d.arcs + a0;
    if (threadIdx.x == 0) S.blk_min = CLD_INF64;
    __syncthreads();
    for (int32_t base = 0; base < a1; base += (int32_t)blockDim.x) {
      const uint64_t cur = S.blk_min;   // the same for every thread: nothing changes it between the barriers
      const int32_t a = base + (int32_t)threadIdx.x;
      if (a < a1) {
        const uint64_t arc = row[a];
        const uint64_t w = arc >> 32;
        if (pull_more(w, cur, delta, next)) {
          const uint64_t c = pull_offer(job, off, arc, delta, next);
          if (c < cur) atomicMin(&S.blk_min, (unsigned long long)c);
        }
      }
      __syncthreads();
      const int32_t nxt = base + (int32_t)blockDim.x;
      const uint64_t cur2 = S.blk_min;
      const bool stop = nxt >= a1 || !pull_more(row[nxt] >> 32, cur2, delta, next);
      __syncthreads();   // every thread has read S.blk_min before the next chunk changes it
      if (stop) break;
    }
    if (threadIdx.x == 0) pull_apply(job, off, v, S.blk_min, next, S, out);
    __syncthreads();
  }
  __syncthreads();
  if (threadIdx.x == 0) { S.mid_cnt = 0; S.big_cnt = 0; }
  __syncthreads();
}

// CLUSTER2, Contract2: u was assigned last iteration at growth distance dl
// (kept in keyn) with label c; every edge with Delta2 - dl < w <= Delta2 is
// the rescaled edge (c, v) of weight dl + w - Delta2.  Rows are sorted by
// weight, so those arcs are one contiguous range.
__device__ uint32_t c2_boundary(const Job &job, const GDesc &d, int64_t off, uint32_t delta2, uint32_t it, int32_t u,
                                Stage &S, const Out *out) {
  const uint32_t dl = (uint32_t)job.keyn[off + u];
  const uint64_t label = job.key[off + u] & 0xffffffffull;
  const int64_t a0 = d.row_ptr[u];
  const int32_t a1 = (int32_t)(d.row_ptr[u + 1] - a0);
  const uint64_t *row = d.arcs + a0;
  int32_t lo = 0, hi = a1;
  while (lo < hi) {   // first arc with w > delta2 - dl
    const int32_t mid = lo + ((hi - lo) >> 1);
    if ((uint32_t)(row[mid] >> 32) <= delta2 - dl) lo = mid + 1; else hi = mid;
  }
  uint32_t scanned = 0;
  for (int32_t a = lo; a < a1; ++a) {
    const uint64_t arc = row[a];
    const uint32_t w = (uint32_t)(arc >> 32);
    if (w > delta2) break;
    ++scanned;
    const int32_t v = (int32_t)(uint32_t)arc;
    const int64_t gv = off + v;
    const uint64_t cand = ((uint64_t)(dl + w - delta2) << 32) | label;
    if (cand < job.key[gv]) {
      const uint64_t old = atomicMin((unsigned long long *)&job.key[gv], (unsigned long long)cand);
      if (atomicExch(&job.fstamp[gv], it) != it) stage_push(S, out, 0, v);
      if (old == CLD_INF64) stage_push(S, out, 1, v);
    }
  }
  return scanned;
}

// Items [a, b) of the index space, all of graph g.
__device__ uint32_t process_run(const Job &job, int g, uint32_t a, uint32_t b, uint32_t it, Stage &S) {
  const GDesc &d = job.desc[g];
  const GState &s = job.st[g];
  GCount &cn = job.cn[g];
  const int64_t off = d.off;
  const uint32_t phase = s.phase;
  const uint32_t delta = s.delta, level_id = s.level_id, stage = s.stage, ucur = s.ucur, theta = s.theta;
  const uint32_t row_lim = row_limit(d, delta, s.row_base);
  const uint32_t theta_row = row_lim < theta ? row_lim : theta;
  const uint32_t fcur = s.fcur, fnxt = s.fnxt, blk = s.blk;
  const uint64_t T = s.T;
  Out o[3] = {};
  int nout = 0;
  switch (phase) {
    case PH_SELECT:
      o[0] = {job.pool[fcur] + off, &cn.cnt[fcur].v};
      o[1] = {job.C + off, &cn.cntC.v};
      nout = 2;
      break;
    case PH_RELAX:
      o[0] = {job.pool[fnxt] + off, &cn.cnt[fnxt].v};
      o[1] = {job.C + off, &cn.cntC.v};
      o[2] = {job.pool[blk] + off, &cn.cnt[blk].v};
      nout = 3;
      break;
    case PH_COMPACT:
      o[0] = {job.U[ucur ^ 1] + off, &cn.cntU[ucur ^ 1].v};
      nout = 1;
      break;
    case PH_MERGE:
      o[0] = {job.pool[fcur] + off, &cn.cnt[fcur].v};
      nout = 1;
      break;
    case PH_PULL:
    case PH_C2_SELECT:
    case PH_C2_BOUNDARY:
      o[0] = {job.pool[fcur] + off, &cn.cnt[fcur].v};
      o[1] = {job.C + off, &cn.cntC.v};
      nout = 2;
      break;
    default:
      break;
  }
  const bool steps = d.variant == CLDIAM_VARIANT_STEPS;
  const bool resume = !steps && !s.c2;   // long rows resume their last scan (keyn/slim hold scan records)
  if (threadIdx.x == 0) {
    S.out[0] = o[0];
    S.out[1] = o[1];
    S.out[2] = o[2];
    S.acc = (phase == PH_NEXT || phase == PH_NEXT_PULL) ? CLD_INF64 : 0ull;
    S.blk_arcs = 0;
    S.acc32 = 0;
    S.fmin = 0xffffffffu;
    S.lq_cnt[0] = 0;
    S.lq_cnt[1] = 0;
    S.mid_cnt = 0;
    S.big_cnt = 0;
  }
  if (phase == PH_RMAX) {
    for (uint32_t t = threadIdx.x; t < kRmaxSlots; t += blockDim.x) {
      S.rmax.tag[t] = kRmaxFree;
      S.rmax.mx[t] = 0;
    }
  }
  __syncthreads();
  const Out *out = S.out;
  uint32_t scanned = 0;
  for (uint32_t r = a; r < b; r += blockDim.x) {
    const uint32_t i = r + threadIdx.x;
    if (i < b) {
      const uint32_t idx = i;
      switch (phase) {
        case PH_SELECT: {
          const int32_t v = job.U[ucur][off + idx];
          if (stage == 0 && d.pull_mode == CLDIAM_PULL_AUTO) {
            const uint32_t deg = (uint32_t)(d.row_ptr[v + 1] - d.row_ptr[v]);
            if (deg > d.hub_deg) atomicAdd(&S.acc, (unsigned long long)deg);
          }
          const uint32_t x0 = cld_philox_word0((uint32_t)v, stage, 0u, 0u, (uint32_t)d.seed, (uint32_t)(d.seed >> 32));
          if ((uint64_t)x0 < T) {
            job.key[off + v] = (uint64_t)(uint32_t)v;
            if (steps) job.keyn[off + v] = (uint64_t)(uint32_t)v;
            stage_push(S, out, 0, v);
            stage_push(S, out, 1, v);
            atomicAdd(&S.acc32, 1u);
          }
          break;
        }
        case PH_RELAX:
          if (steps)
            scanned += relax_sync(job, d, off, delta, it, level_id, job.pool[fcur][off + idx], S, out);
          else
            scanned += relax_item(job, d, off, delta, theta, theta_row, it, level_id, job.pool[fcur][off + idx], S,
                                  out, &S.lq_cnt[0], S.lq[0]);
          break;
        case PH_COMMIT: {
          const int32_t v = job.pool[fnxt][off + idx];
          job.key[off + v] = job.keyn[off + v];
          break;
        }
        case PH_MERGE: {
          const int32_t u = job.pool[blk][off + idx];
          if (atomicExch(&job.fstamp[off + u], s.fid) != s.fid) stage_push(S, out, 0, u);
          break;
        }
        case PH_C2_INIT:
          job.key[off + idx] = CLD_INF64;
          job.U[0][off + idx] = (int32_t)idx;
          break;
        case PH_C2_SELECT: {
          const int32_t v = job.U[ucur][off + idx];
          const uint32_t x0 =
              cld_philox_word0((uint32_t)v, stage + 1, 0u, 1u, (uint32_t)d.seed, (uint32_t)(d.seed >> 32));
          if ((uint64_t)x0 < T) {
            job.key[off + v] = (uint64_t)(uint32_t)v;
            job.R[off + v] = stage + 1;   // birth iteration of the center
            stage_push(S, out, 0, v);
            stage_push(S, out, 1, v);
            atomicAdd(&S.acc32, 1u);
          }
          break;
        }
        case PH_C2_BOUNDARY:
          scanned += c2_boundary(job, d, off, delta, it, job.pool[blk][off + idx], S, out);
          break;
        case PH_C2_ASSIGN: {
          const int32_t v = job.U[ucur][off + idx];
          const uint64_t k = job.key[off + v];
          if (k == CLD_INF64) break;
          const uint32_t c = (uint32_t)k;
          const uint64_t local = k >> 32;
          const uint64_t Dv = local + (uint64_t)delta * (uint64_t)(stage + 1 - job.R[off + c]);
          d.cluster[v] = (int32_t)c;
          d.D[v] = Dv;
          job.keyn[off + v] = local;   // kept for next iteration's rescaled edges
          job.key[off + v] = (uint64_t)c;
          if (Dv > S.acc) atomicMax(&S.acc, (unsigned long long)Dv);
          break;
        }
        case PH_NEXT: {
          const int32_t u = job.pool[blk][off + idx];
          const int32_t deg = (int32_t)(d.row_ptr[u + 1] - d.row_ptr[u]);
          if (deg > d.mid_deg && defer_row(S, u, deg, d.big_deg)) break;
          const uint64_t best = next_small(job, d, off, delta, u);
          if (best < S.acc) atomicMin(&S.acc, (unsigned long long)best);
          break;
        }
        case PH_PULL:
        case PH_NEXT_PULL:
          pull_item(job, d, off, delta, job.U[ucur][off + idx], phase == PH_NEXT_PULL, S, out);
          break;
        case PH_ASSIGN: {
          // over the stage's uncovered list (in node order at the first
          // stage, so these reads and writes are coalesced); covered nodes
          // are the ones with a finite key
          const int32_t v = job.U[ucur][off + idx];
          const uint64_t k = job.key[off + v];
          if (k == CLD_INF64) break;
          const uint32_t c = (uint32_t)k;
          const uint64_t Dv = (k >> 32) + job.R[off + c];
          d.cluster[v] = (int32_t)c;
          d.D[v] = Dv;
          if (Dv > S.acc) atomicMax(&S.acc, (unsigned long long)Dv);
          break;
        }
        case PH_RMAX: {
          const int32_t v = job.U[ucur][off + idx];
          const uint64_t k = job.key[off + v];
          if (k == CLD_INF64) break;
          const uint32_t c = (uint32_t)k;
          const uint64_t Dv = d.D[v];
          // a stage has few clusters: fold the maxima in LDS first (the slot
          // of c, once claimed by c), in global memory when another center
          // holds the slot
          const uint32_t slot = (c * 2654435761u) >> 22;   // 10 bits: kRmaxSlots
          uint32_t t = S.rmax.tag[slot];
          if (t == kRmaxFree) {
            t = atomicCAS(&S.rmax.tag[slot], kRmaxFree, c);
            if (t == kRmaxFree) t = c;
          }
          if (t == c) {
            if (Dv > S.rmax.mx[slot]) atomicMax(&S.rmax.mx[slot], (unsigned long long)Dv);
          } else {
            uint64_t *rr = &job.R[off + c];
            if (Dv > *rr) atomicMax((unsigned long long *)rr, (unsigned long long)Dv);
          }
          job.key[off + v] = (uint64_t)c;
          job.keyn[off + v] = (uint64_t)c;
          break;
        }
        case PH_COMPACT: {
          const int32_t v = job.U[ucur][off + idx];
          if (job.key[off + v] == CLD_INF64) stage_push(S, out, 0, v);
          break;
        }
        case PH_SINGLE: {
          const int32_t v = job.U[ucur][off + idx];
          d.cluster[v] = v;
          d.D[v] = 0;
          break;
        }
        default:
          break;
      }
    }
    if (phase == PH_PULL || phase == PH_NEXT_PULL) pull_rows(job, d, off, delta, phase == PH_NEXT_PULL, S, out);
    if (phase == PH_RELAX || phase == PH_NEXT)
      scanned += coop_rows(job, d, off, delta, it, level_id, S, out, steps ? nullptr : &S.lq_cnt[0],
                           steps ? nullptr : S.lq[0], phase == PH_NEXT ? 1 : (steps ? 2 : 0), resume);
    if (nout) {
      __syncthreads();
      if (threadIdx.x < (unsigned)nout && S.cnt[threadIdx.x] > kStageCap - kSweepThreads) S.flush = 1;
      __syncthreads();
      if (S.flush) stage_flush(S, out, nout);
    }
  }
  if (phase == PH_RELAX && steps && scanned) atomicAdd(&S.acc, (unsigned long long)scanned);
  if (phase == PH_RELAX && !steps) {
    // Local rounds: keep relaxing the neighbours this workgroup improved.
    // Every improved node is also on the global next frontier, so these
    // rounds only move the fixpoint closer; dropped overflow loses nothing.
    int q = 0;
    // a small frontier leaves the grid idle between sweeps: let each
    // workgroup carry its part of the growth further before the next one
    const uint32_t graph_items = job.seg[2 * job.G + 1 + g];
    const int rounds = (d.local_rounds > 0 && graph_items <= kSmallFrontier && d.local_rounds < kSmallRounds)
                           ? kSmallRounds : d.local_rounds;
    for (int round = 0; round < rounds; ++round) {
      if (threadIdx.x == 0)
        S.stop = job.cutoff < (uint32_t)job.nblocks &&
                 __hip_atomic_load(&job.ctl->idle.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= job.cutoff;
      __syncthreads();
      const uint32_t n = S.lq_cnt[q] < d.lq_cap ? S.lq_cnt[q] : d.lq_cap;
      if (n == 0 || S.stop) break;
      if (threadIdx.x == 0) S.lq_cnt[q ^ 1] = 0;
      __syncthreads();
      for (uint32_t t = threadIdx.x; t < n; t += blockDim.x)
        scanned += relax_item(job, d, off, delta, theta, theta_row, it, level_id, S.lq[q][t], S, out,
                              &S.lq_cnt[q ^ 1], S.lq[q ^ 1]);
      scanned += coop_rows(job, d, off, delta, it, level_id, S, out, &S.lq_cnt[q ^ 1], S.lq[q ^ 1], 0, resume);
      __syncthreads();
      if (threadIdx.x < (unsigned)nout && S.cnt[threadIdx.x] > kStageCap - kSweepThreads) S.flush = 1;
      __syncthreads();
      if (S.flush) stage_flush(S, out, nout);
      q ^= 1;
    }
  }
  if (nout) stage_flush(S, out, nout);
  __syncthreads();
  if (phase == PH_RMAX) {
    for (uint32_t t = threadIdx.x; t < kRmaxSlots; t += blockDim.x) {
      const uint32_t c = S.rmax.tag[t];
      if (c == kRmaxFree) continue;
      uint64_t *rr = &job.R[off + c];
      const unsigned long long m = S.rmax.mx[t];
      if (m > *rr) atomicMax((unsigned long long *)rr, m);
    }
  }
  if (threadIdx.x == 0) {
    if ((phase == PH_NEXT || phase == PH_NEXT_PULL) && S.acc != CLD_INF64) atomicMin(&cn.next.v, S.acc);
    if ((phase == PH_ASSIGN || phase == PH_C2_ASSIGN) && S.acc) atomicMax(&cn.radius.v, S.acc);
    if ((phase == PH_SELECT || phase == PH_C2_SELECT) && S.acc32) atomicAdd(&cn.centers.v, S.acc32);
    if (phase == PH_SELECT && S.acc) atomicAdd(&cn.hub_arcs.v, S.acc);
    if (phase == PH_RELAX && S.fmin != 0xffffffffu) atomicMin(&cn.fmin.v, S.fmin);
    if (phase == PH_RELAX && steps && S.acc) atomicAdd(&cn.msgs.v, S.acc);
    if (phase == PH_RELAX && S.blk_arcs) atomicAdd(&cn.blk_arcs.v, S.blk_arcs);
  }
  __syncthreads();
  return scanned;
}

// Chunk index -> graph (largest g with seg[g] <= i).
__device__ __forceinline__ int graph_of(const Job &job, uint32_t i) {
  int lo = 0, hi = job.G - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (job.seg[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The sweep's work is a list of chunks, each a range of one graph's items
// (at most one chunk of a graph per workgroup); workgroup b takes chunks b,
// b + nblocks, ...
__device__ void sweep(const Job &job, uint32_t block, uint32_t nblocks, Stage &S) {
  const uint32_t total = job.ctl->total;
  const uint32_t it = job.ctl->sweep_id;
  if (threadIdx.x < 3) S.cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) S.flush = 0;
  __syncthreads();
  uint32_t scanned = 0;
  // chunk b first; chunks past the first nblocks go to whichever workgroup
  // asks next, so that costly chunks (hub rows) do not hold up a sweep
  for (uint32_t v = block; v < total;) {
    const int g = graph_of(job, v);
    const uint32_t per = job.seg[job.G + 1 + g];
    const uint32_t n_items = job.seg[2 * job.G + 1 + g];
    const uint32_t lo = (v - job.seg[g]) * per;
    const uint32_t hi = lo + per < n_items ? lo + per : n_items;
    scanned += process_run(job, g, lo, hi, it, S);
    if (total <= nblocks) break;
    if (threadIdx.x == 0) S.chunk = nblocks + atomicAdd(&job.ctl->cursor.v, 1u);
    __syncthreads();
    v = S.chunk;
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(&job.ctl->idle.v, 1u);
  for (int o = 32; o >= 1; o >>= 1) scanned += __shfl_xor(scanned, o);
  if (cld_lane() == 0 && scanned) atomicAdd(&job.ctl->arcs.v, (unsigned long long)scanned);
}

// ---------------------------------------------------------------- kernels --

__global__ void __launch_bounds__(256) k_init(Job job, int64_t total_n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total_n; i += stride) {
    job.key[i] = CLD_INF64;
    job.keyn[i] = CLD_INF64;
    job.slim[i] = 0;
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

// Fresh state for one graph of a server job (node range [off, off + n)).
__global__ void __launch_bounds__(256) k_init_range(Job job, int64_t off, int32_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;

  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    job.key[off + i] = CLD_INF64;
    job.keyn[off + i] = CLD_INF64;
    job.slim[off + i] = 0;
    job.R[off + i] = 0;
    job.fstamp[off + i] = 0;
    job.bstamp[off + i] = 0;
    job.U[0][off + i] = (int32_t)i;
  }
}

// A job of up to kSmallControl graphs takes a one-wave control step: no
// cross-wave barriers, a 64-entry scan.
template <int T>
__global__ void __launch_bounds__(T) k_control(Job job) { control_block<T>(job); }

constexpr int kSmallControl = 64;

void launch_control(const Job &job, hipStream_t stream) {
  if (job.G <= kSmallControl) k_control<kSmallControl><<<1, kSmallControl, 0, stream>>>(job);
  else k_control<kThreads><<<1, kThreads, 0, stream>>>(job);
}

__global__ void __launch_bounds__(kSweepThreads) k_sweep(Job job) {
  __shared__ Stage S;
  if (job.ctl->done) return;
  sweep(job, blockIdx.x, gridDim.x, S);
}

__global__ void __launch_bounds__(kSweepThreads) k_persistent(Job job) {
  __shared__ Stage S;
  const uint32_t nb = gridDim.x;
  for (;;) {
    if (blockIdx.x == 0) control_block<kSweepThreads>(job);
    if (!cld_grid_barrier(&job.ctl->bar, &job.ctl->timeout, nb)) return;
    if (job.ctl->done || job.ctl->timeout) return;
    sweep(job, blockIdx.x, nb, S);
    if (!cld_grid_barrier(&job.ctl->bar, &job.ctl->timeout, nb)) return;
  }
}

// ------------------------------------------------------------------- host --

struct Layout {
  GDesc *desc;
  GState *st;
  GCount *cn;
  Ctl *ctl;
  uint32_t *seg;
  int32_t *log;
  uint64_t *key, *keyn, *R;
  uint32_t *slim, *fstamp, *bstamp;
  int32_t *pool[3], *U[2], *C;
};

template <class A>
bool carve(A &a, int64_t N, int32_t G, Layout *L) {
  auto p_desc = a.template take<GDesc>(G);
  auto p_st = a.template take<GState>(G);
  auto p_cn = a.template take<GCount>(G);
  auto p_ctl = a.template take<Ctl>(1);
  auto p_seg = a.template take<uint32_t>(3 * (size_t)G + 1);
  auto p_log = a.template take<int32_t>((size_t)G * CLDIAM_STAGE_LOG * 4);
  auto p_key = a.template take<uint64_t>(N);
  auto p_keyn = a.template take<uint64_t>(N);
  auto p_R = a.template take<uint64_t>(N);
  auto p_slim = a.template take<uint32_t>(N);
  auto p_fs = a.template take<uint32_t>(N);
  auto p_bs = a.template take<uint32_t>(N);
  auto p0 = a.template take<int32_t>(N);
  auto p1 = a.template take<int32_t>(N);
  auto p2 = a.template take<int32_t>(N);
  auto u0 = a.template take<int32_t>(N);
  auto u1 = a.template take<int32_t>(N);
  auto c = a.template take<int32_t>(N);
  if (L) {
    *L = Layout{(GDesc *)p_desc, (GState *)p_st, (GCount *)p_cn, (Ctl *)p_ctl, (uint32_t *)p_seg, (int32_t *)p_log,
                (uint64_t *)p_key, (uint64_t *)p_keyn, (uint64_t *)p_R, (uint32_t *)p_slim, (uint32_t *)p_fs,
                (uint32_t *)p_bs,
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

constexpr size_t kMirrorOffset = cld::kPinnedBytes - 128;   // host-loop mirror words in the readback buffer
constexpr uint32_t kLeadSteps = 16;   // control + sweep steps the host queues ahead of the device
static_assert(sizeof(Ctl) <= kMirrorOffset, "control block and mirror words must fit a pooled pinned buffer");

// Workgroups of the sweep grid: one per CU unless requested (bounded by the
// co-resident maximum for the persistent kernel).
int grid_blocks(int driver, int requested, int *blocks) {
  int coop_blocks = 0;
  int rc = cld::cooperative_blocks((const void *)k_persistent, kSweepThreads, kCuThreads / kSweepThreads,
                                   &coop_blocks);
  if (rc) return rc;
  int dev = 0, cus = 0;
  CLD_HIP(hipGetDevice(&dev));
  CLD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  int want = requested > 0 ? requested : cus * (kCuThreads / kSweepThreads);
  if (driver == CLDIAM_DRIVER_HOST) {
    *blocks = want;
    return CLDIAM_OK;
  }
  if (coop_blocks == 0) {
    *blocks = 0;
    return CLDIAM_OK;
  }
  *blocks = want < coop_blocks ? want : coop_blocks;
  return CLDIAM_OK;
}

// Finished workgroups after which the others end their local rounds.
uint32_t local_cutoff(const cldiam_tuning *tuning, int blocks) {
  int pct = tuning && tuning->local_cutoff > 0 ? tuning->local_cutoff : kLocalCutoffPct;
  if (pct > 100) pct = 100;
  return (uint32_t)(((int64_t)pct * blocks + 99) / 100);
}

// Descriptor of one graph (node offset set by the caller); returns a status.
int make_desc(const cldiam_graph &x, int g, const cldiam_tuning *tuning, GDesc *out) {
  float bucket_width = tuning ? tuning->bucket_width : 0.f;
  if (x.n < 1 || x.m < 0 || x.m >= ((int64_t)1 << 40) || !x.d_row_ptr || (x.m && !x.d_arcs) || !x.d_cluster ||
      !x.d_D || x.params.tau < 1) {
    cld::set_error("decompose: invalid graph %d (n=%d m=%lld tau=%u)", g, x.n, (long long)x.m, x.params.tau);
    return CLDIAM_EINVAL;
  }
  GDesc &d = *out;
  memset(&d, 0, sizeof d);
  d.row_ptr = x.d_row_ptr;
  d.arcs = x.d_arcs;
  d.cluster = x.d_cluster;
  d.D = x.d_D;
  d.n = x.n;
  const double gamma = 4.0 * M_LN2;
  const double L = log2((double)x.n);
  d.K = gamma * x.params.tau * L;
  d.stop = (uint32_t)ceil(8.0 * x.params.tau * L);
  d.seed = x.params.seed;
  if (x.params.variant > CLDIAM_VARIANT_CLUSTER2) {
    cld::set_error("decompose: unknown variant %u (graph %d)", x.params.variant, g);
    return CLDIAM_EINVAL;
  }
  d.variant = x.params.variant;
  d.step_cap = x.params.step_cap;
  // local rounds: the caller's, else many on sparse graphs (long growth
  // paths: each round carries the frontier one more hop without a sweep)
  // and few on dense ones (their rows are long and their growth shallow)
  // long-row bucket: the caller's shift, else the default; none for
  // synchronous steps (their sweeps take every active node)
  // The default narrows with the graph: a narrower bucket saves rescans of
  // long rows but costs sweeps, whose fixed cost weighs more on small graphs.
  const int32_t rs = tuning ? tuning->row_bucket_shift : 0;
  int32_t auto_shift = 0;
  while (auto_shift < 62 && (x.m >> (auto_shift + 1)) > 0) ++auto_shift;   // floor(log2 m)
  auto_shift = auto_shift / 2 - 6;
  auto_shift = auto_shift < kRowShiftMin ? kRowShiftMin : (auto_shift > kRowShiftMax ? kRowShiftMax : auto_shift);
  d.row_shift = (rs < 0 || d.variant == CLDIAM_VARIANT_STEPS) ? -1 : (rs == 0 ? auto_shift : (rs > 31 ? 31 : rs));
  // large dense graphs: the cost of a chunk varies with the hub rows it
  // holds, so cut their frontiers finer and hand the chunks out on demand
  const int32_t cf = tuning ? tuning->chunk_factor : 0;
  d.chunk_factor = cf > 0 ? (cf > 64 ? 64 : cf)
                          : ((x.m > (int64_t)kDenseDegree * x.n && x.n > kDenseLarge) ? kDenseChunks : 1);
  // row tiers (threads per row) and the local queue's size
  const int32_t wr = tuning ? tuning->wave_row_min : 0, gr = tuning ? tuning->group_row_min : 0;
  const int32_t lqc = tuning ? tuning->local_queue : 0;
  const bool dense = x.m > (int64_t)kDenseDegree * x.n;
  d.mid_deg = wr > 0 ? (wr > (1 << 20) ? (1 << 20) : wr) : (dense ? kDenseWaveRow : kMidDeg);
  d.big_deg = gr > 0 ? (gr > (1 << 30) ? (1 << 30) : gr) : kBigDeg;
  if (d.big_deg < d.mid_deg) d.big_deg = d.mid_deg;
  d.lq_cap = lqc > 0 ? (uint32_t)(lqc < 64 ? 64 : (lqc > kLocalCap ? kLocalCap : lqc)) : (uint32_t)kLocalCap;
  const int32_t pm = tuning ? tuning->pull_mode : 0;
  if (pm < 0 || pm > CLDIAM_PULL_ALWAYS) {
    cld::set_error("decompose: unknown pull mode %d (graph %d)", pm, g);
    return CLDIAM_EINVAL;
  }
  // CLUSTER2 (its preliminary CLUSTER run included) and the literal steps never pull
  d.pull_mode = d.variant == CLDIAM_VARIANT_FIXPOINT ? (uint32_t)pm : (uint32_t)CLDIAM_PULL_NEVER;
  {
    const int64_t hd = x.m / x.n * kHubDegree;
    d.hub_deg = (uint32_t)(hd < 0xffffffffll ? hd : 0xffffffffll);
    d.hub_min = (uint64_t)(x.m / kHubShare);
  }
  if (tuning && tuning->local_rounds >= 0) d.local_rounds = tuning->local_rounds > 64 ? 64 : tuning->local_rounds;
  else if (x.m <= (int64_t)kDenseDegree * x.n) d.local_rounds = kLocalRounds;
  else d.local_rounds = x.n > kDenseLarge ? kLocalRoundsDense : 0;
  d.c2_iters = 0;
  while (((int64_t)1 << d.c2_iters) < (int64_t)x.n) d.c2_iters++;   // ceil(log2 n)
  uint64_t d0 = x.params.delta0;
  if (d0 == 0) d0 = x.m > 0 ? x.weight_sum / (uint64_t)x.m : 1;
  if (d0 < 1) d0 = 1;
  if (d0 > CLD_DELTA_MAX) {
    cld::set_error("decompose: initial Delta %llu above 2^31 (graph %d)", (unsigned long long)d0, g);
    return CLDIAM_EOVERFLOW;
  }
  d.delta0 = (uint32_t)d0;
  // bucket width in mean arc weights -> distance units (0 = unbounded)
  if (bucket_width == 0.f) bucket_width = CLDIAM_BUCKET_DEFAULT;
  d.bucket = 0;
  if (bucket_width > 0.f && x.m > 0 && d.variant != CLDIAM_VARIANT_STEPS) {
    const double b = ceil((double)bucket_width * ((double)x.weight_sum / (double)x.m));
    d.bucket = b >= 4294967295.0 ? 0u : (b < 1.0 ? 1u : (uint32_t)b);
  }
  return CLDIAM_OK;
}

void fill_stats(const GDesc &d, const GState &st, const GCount &cn, const int32_t *log, cldiam_stats *o) {
  memset(o, 0, sizeof *o);
  o->stages = (int32_t)st.stage;
  o->levels = (int32_t)st.levels;
  o->delta0 = d.delta0;
  o->delta_end = st.delta;
  o->stop = (int32_t)d.stop;
  o->num_clusters = (int32_t)(st.centers_total + st.singletons);
  o->singletons = (int32_t)st.singletons;
  o->sweeps = (int32_t)st.sweeps;
  o->radius = cn.radius.v;
  o->status = st.status;
  o->rounds = st.rounds;
  o->radius1 = st.radius1;
  o->updates = st.updates;
  o->messages = cn.msgs.v;
  for (int s = 0; s < CLDIAM_STAGE_LOG && s < o->stages; ++s) {
    const int32_t *l = log + (size_t)s * 4;
    o->stage_uncovered[s] = l[0];
    o->stage_centers[s] = l[1];
    o->stage_covered[s] = l[2];
    o->stage_delta[s] = (uint32_t)l[3];
  }
}

int read_wall_limit(unsigned long long *limit) {
  int dev = 0, khz = 0;
  CLD_HIP(hipGetDevice(&dev));
  CLD_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) khz = 100000;
  *limit = (unsigned long long)khz * 1000ull * kJobSeconds;
  return CLDIAM_OK;
}

}  // namespace

extern "C" size_t cldiam_decompose_workspace_size(int64_t total_n, int32_t num_graphs) {
  if (total_n < 1 || num_graphs < 1) return 0;
  SizeArena s;
  carve(s, total_n, num_graphs, nullptr);
  return s.s.used;
}

extern "C" int cldiam_decompose_batch(int32_t G, const cldiam_graph *gs, cldiam_stats *stats, int driver,
                                      const cldiam_tuning *tuning, void *ws, size_t ws_bytes, void *stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (G < 1 || !gs) { cld::set_error("decompose: num_graphs < 1 or no graphs"); return CLDIAM_EINVAL; }
  int64_t N = 0;
  std::vector<GDesc> desc(G);
  for (int g = 0; g < G; ++g) {
    int rc = make_desc(gs[g], g, tuning, &desc[g]);
    if (rc) return rc;
    desc[g].off = N;
    N += gs[g].n;
  }
  if (N >= ((int64_t)1 << 31)) { cld::set_error("decompose: more than 2^31 nodes in one job"); return CLDIAM_EINVAL; }
  Layout L;
  PtrArena pa(ws, ws_bytes);
  if (!carve(pa, N, G, &L) || pa.a.used > ws_bytes) {
    cld::set_error("decompose: workspace of %zu bytes, %zu needed", ws_bytes, cldiam_decompose_workspace_size(N, G));
    return CLDIAM_ENOMEM;
  }
  Job job{};
  job.desc = L.desc; job.st = L.st; job.cn = L.cn; job.ctl = L.ctl; job.seg = L.seg; job.log = L.log;
  job.key = L.key; job.keyn = L.keyn; job.R = L.R; job.slim = L.slim; job.fstamp = L.fstamp;
  job.bstamp = L.bstamp;
  for (int i = 0; i < 3; ++i) job.pool[i] = L.pool[i];
  job.U[0] = L.U[0]; job.U[1] = L.U[1]; job.C = L.C; job.G = G;

  CLD_HIP(hipMemcpyAsync(L.desc, desc.data(), sizeof(GDesc) * G, hipMemcpyHostToDevice, stream));
  CLD_HIP(hipMemsetAsync(L.st, 0, sizeof(GState) * G, stream));
  CLD_HIP(hipMemsetAsync(L.cn, 0, sizeof(GCount) * G, stream));
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
  k_init<<<cld::blocks_for(N, 256, 8192), 256, 0, stream>>>(job, N);
  CLD_LAUNCH_CHECK("k_init");

  int blocks = 0;
  {
    int rc = grid_blocks(driver == CLDIAM_DRIVER_PERSISTENT ? driver : CLDIAM_DRIVER_HOST,
                         tuning ? tuning->grid_blocks : 0, &blocks);
    if (rc) return rc;
    if (blocks == 0 && driver == CLDIAM_DRIVER_PERSISTENT) {
      cld::set_error("decompose: device has no cooperative launch");
      return CLDIAM_EINVAL;
    }
  }
  const bool persistent = driver == CLDIAM_DRIVER_PERSISTENT && blocks > 0;
  if (!persistent && blocks <= 0) blocks = 256;
  if (blocks > 65535) blocks = 65535;
  job.nblocks = blocks;
  job.cutoff = local_cutoff(tuning, blocks);
  cld::Pinned<Ctl> pinned;   // readback buffer, back to the pool when the call returns
  Ctl *hc = pinned.p;
  if (!hc) { cld::set_error("decompose: pinned host buffer allocation failed"); return CLDIAM_EHIP; }
  // the last line of the same buffer: the control step's mirror for the host loop
  volatile uint32_t *hm = (volatile uint32_t *)((char *)hc + kMirrorOffset);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  CLD_HIP(hipEventCreate(&ev0));
  CLD_HIP(hipEventCreate(&ev1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() { if (a) (void)hipEventDestroy(a); if (b) (void)hipEventDestroy(b); }
  } evg{ev0, ev1};
  CLD_HIP(hipEventRecord(ev0, stream));
  if (persistent) {
    void *args[] = {&job};
    CLD_HIP(hipLaunchCooperativeKernel((const void *)k_persistent, dim3(blocks), dim3(kSweepThreads), args, 0,
                                       stream));
    CLD_HIP(hipEventRecord(ev1, stream));
    CLD_HIP(hipMemcpyAsync(hc, L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    CLD_HIP(hipStreamSynchronize(stream));
    if (hc->timeout) { cld::set_error("decompose: grid barrier timed out"); return CLDIAM_ETIMEOUT; }
    if (!hc->done && !hc->error) { cld::set_error("decompose: persistent kernel ended early"); return CLDIAM_EHIP; }
  } else {
    // The host queues control + sweep steps at most kLeadSteps ahead of the
    // control steps the device has finished (read from the mapped mirror, no
    // stream synchronisation), and stops queueing once the device reports the
    // job done: only the steps already queued then run, and they return at once.
    hm[0] = 0;
    hm[1] = 0;
    uint32_t *dm = nullptr;
    CLD_HIP(hipHostGetDevicePointer((void **)&dm, (void *)hm, 0));
    job.hmirror = dm;
    const auto t0 = std::chrono::steady_clock::now();
    uint32_t queued = 0;
    for (;;) {
      if (hm[1]) break;
      if (queued < hm[0] + kLeadSteps) {
        launch_control(job, stream);
        k_sweep<<<blocks, kSweepThreads, 0, stream>>>(job);
        ++queued;
        if ((queued & 15u) == 0) CLD_LAUNCH_CHECK("k_sweep");
        continue;
      }
      if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(kJobSeconds + 30)) {
        CLD_HIP(hipStreamSynchronize(stream));
        cld::set_error("decompose: host-driven job exceeded its time limit");
        return CLDIAM_ETIMEOUT;
      }
      std::this_thread::yield();
    }
    CLD_LAUNCH_CHECK("k_sweep");
    CLD_HIP(hipEventRecord(ev1, stream));
    CLD_HIP(hipMemcpyAsync(hc, L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    CLD_HIP(hipStreamSynchronize(stream));
    if (!hc->done) { cld::set_error("decompose: host-driven job ended without its done flag"); return CLDIAM_EHIP; }
    blocks = 0;
  }
  std::vector<GState> st(G);
  std::vector<GCount> cn(G);
  std::vector<int32_t> lg((size_t)G * CLDIAM_STAGE_LOG * 4);
  CLD_HIP(hipMemcpyAsync(st.data(), L.st, sizeof(GState) * G, hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipMemcpyAsync(cn.data(), L.cn, sizeof(GCount) * G, hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipMemcpyAsync(lg.data(), L.log, sizeof(int32_t) * lg.size(), hipMemcpyDeviceToHost, stream));
  CLD_HIP(hipStreamSynchronize(stream));
  float kernel_ms = 0.f;
  CLD_HIP(hipEventElapsedTime(&kernel_ms, ev0, ev1));
  int rc = CLDIAM_OK;
  for (int g = 0; g < G; ++g) {
    if (st[g].status != CLDIAM_OK && rc == CLDIAM_OK) {
      rc = st[g].status;
      cld::set_error("decompose: graph %d failed: %s", g, cldiam_strerror(rc));
    }
    if (!stats) continue;
    fill_stats(desc[g], st[g], cn[g], &lg[(size_t)g * CLDIAM_STAGE_LOG * 4], &stats[g]);
    stats[g].arcs_scanned = (G == 1) ? hc->arcs.v : 0;
    stats[g].grid_blocks = blocks;
    stats[g].kernel_ms = kernel_ms;
    stats[g].iterations = (int32_t)hc->iterations;
  }
  if (rc == CLDIAM_OK && hc->error) {
    rc = -(int)hc->error;
    cld::set_error("decompose: device reported %s", cldiam_strerror(rc));
  }
  return rc;
}

extern "C" int cldiam_decompose(const cldiam_graph *g, cldiam_stats *stats, int driver, const cldiam_tuning *tuning,
                                void *ws, size_t ws_bytes, void *stream) {
  return cldiam_decompose_batch(1, g, stats, driver, tuning, ws, ws_bytes, stream);
}

// ----------------------------------------------------------- server job --
// A long-lived decomposition job with graph slots: requests are queued by
// cldiam_server_submit, admitted between sweeps when a slot and a node range
// of the workspace are free, advanced together with every other active graph,
// and released as soon as they finish.

struct cldiam_server {
  Layout L;
  Job job;
  int64_t ncap;
  int32_t gcap;
  cldiam_tuning tuning;
  hipStream_t stream;
  int blocks;
  std::vector<GDesc> desc;
  std::vector<uint64_t> tag;
  std::vector<char> active;
  std::vector<std::pair<int64_t, int64_t>> free_ranges;  // (offset, length), sorted by offset
  struct Pending {
    GDesc d;
    uint64_t tag;
  };
  std::vector<Pending> queue;
  size_t qhead = 0;
  struct Done {
    uint64_t tag;
    cldiam_stats st;
  };
  std::vector<Done> done;
  std::vector<GState> st_host;
  Ctl *hc = nullptr;
};

namespace {

bool take_range(cldiam_server *s, int64_t n, int64_t *off) {
  for (size_t i = 0; i < s->free_ranges.size(); ++i) {
    auto &r = s->free_ranges[i];
    if (r.second >= n) {
      *off = r.first;
      r.first += n;
      r.second -= n;
      if (r.second == 0) s->free_ranges.erase(s->free_ranges.begin() + i);
      return true;
    }
  }
  return false;
}

void give_range(cldiam_server *s, int64_t off, int64_t n) {
  auto &fr = s->free_ranges;
  auto it = std::lower_bound(fr.begin(), fr.end(), std::make_pair(off, (int64_t)0));
  it = fr.insert(it, {off, n});
  size_t i = it - fr.begin();
  if (i + 1 < fr.size() && fr[i].first + fr[i].second == fr[i + 1].first) {
    fr[i].second += fr[i + 1].second;
    fr.erase(fr.begin() + i + 1);
  }
  if (i > 0 && fr[i - 1].first + fr[i - 1].second == fr[i].first) {
    fr[i - 1].second += fr[i].second;
    fr.erase(fr.begin() + i);
  }
}

}  // namespace

extern "C" size_t cldiam_server_workspace_size(int64_t node_capacity, int32_t max_graphs) {
  return cldiam_decompose_workspace_size(node_capacity, max_graphs);
}

extern "C" int cldiam_server_create(cldiam_server **out, int64_t node_capacity, int32_t max_graphs,
                                    const cldiam_tuning *tuning, void *ws, size_t ws_bytes, void *stream) {
  if (!out || node_capacity < 1 || node_capacity >= ((int64_t)1 << 31) || max_graphs < 1 || max_graphs > 65536) {
    cld::set_error("server: invalid capacity");
    return CLDIAM_EINVAL;
  }
  *out = nullptr;
  cldiam_server *s = new cldiam_server();
  PtrArena pa(ws, ws_bytes);
  if (!carve(pa, node_capacity, max_graphs, &s->L) || pa.a.used > ws_bytes) {
    delete s;
    cld::set_error("server: workspace of %zu bytes, %zu needed", ws_bytes,
                   cldiam_decompose_workspace_size(node_capacity, max_graphs));
    return CLDIAM_ENOMEM;
  }
  s->ncap = node_capacity;
  s->gcap = max_graphs;
  s->tuning = tuning ? *tuning : cldiam_tuning{-1, 0, 0.f, 0, 0, 0, 0, 0, 0, 0};
  s->stream = (hipStream_t)stream;
  Job &job = s->job;
  const Layout &L = s->L;
  job.desc = L.desc; job.st = L.st; job.cn = L.cn; job.ctl = L.ctl; job.seg = L.seg; job.log = L.log;
  job.key = L.key; job.keyn = L.keyn; job.R = L.R; job.slim = L.slim; job.fstamp = L.fstamp;
  job.bstamp = L.bstamp;
  for (int i = 0; i < 3; ++i) job.pool[i] = L.pool[i];
  job.U[0] = L.U[0]; job.U[1] = L.U[1]; job.C = L.C; job.G = max_graphs;
  int rc = grid_blocks(CLDIAM_DRIVER_HOST, tuning ? tuning->grid_blocks : 0, &s->blocks);
  if (rc) { delete s; return rc; }
  if (s->blocks <= 0) s->blocks = 256;
  job.nblocks = s->blocks;
  job.cutoff = local_cutoff(tuning, s->blocks);
  s->desc.assign(max_graphs, GDesc{});
  s->tag.assign(max_graphs, 0);
  s->active.assign(max_graphs, 0);
  s->free_ranges.push_back({0, node_capacity});
  s->st_host.assign(max_graphs, GState{});
  for (auto &g : s->st_host) g.phase = PH_IDLE;
  void *p = nullptr;
  if (hipHostMalloc(&p, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
    delete s;
    cld::set_error("server: pinned host buffer allocation failed");
    return CLDIAM_EHIP;
  }
  s->hc = (Ctl *)p;
  unsigned long long limit = 0;
  rc = read_wall_limit(&limit);
  if (rc) { cldiam_server_destroy(s); return rc; }
  hipStream_t st = s->stream;
  if (hipMemcpyAsync(L.desc, s->desc.data(), sizeof(GDesc) * max_graphs, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(L.st, s->st_host.data(), sizeof(GState) * max_graphs, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemsetAsync(L.cn, 0, sizeof(GCount) * max_graphs, st) != hipSuccess ||
      hipMemsetAsync(L.ctl, 0, sizeof(Ctl), st) != hipSuccess ||
      hipMemcpyAsync(&L.ctl->t_limit, &limit, sizeof limit, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    cldiam_server_destroy(s);
    cld::set_error("server: initialisation failed");
    return CLDIAM_EHIP;
  }
  *out = s;
  return CLDIAM_OK;
}

extern "C" void cldiam_server_destroy(cldiam_server *s) {
  if (!s) return;
  if (s->hc) (void)hipHostFree(s->hc);
  delete s;
}

extern "C" int cldiam_server_submit(cldiam_server *s, const cldiam_graph *g, uint64_t tag) {
  if (!s || !g) { cld::set_error("server: null argument"); return CLDIAM_EINVAL; }
  if (g->n > s->ncap) { cld::set_error("server: graph of %d nodes above the capacity %lld", g->n, (long long)s->ncap); return CLDIAM_ENOMEM; }
  cldiam_server::Pending p;
  int rc = make_desc(*g, 0, &s->tuning, &p.d);
  if (rc) return rc;
  p.tag = tag;
  s->queue.push_back(p);
  return CLDIAM_OK;
}

extern "C" int cldiam_server_step(cldiam_server *s, int32_t max_sweeps, int32_t *h_active, int32_t *h_queued) {
  if (!s || max_sweeps < 0) { cld::set_error("server: invalid step"); return CLDIAM_EINVAL; }
  hipStream_t stream = s->stream;
  Job &job = s->job;
  // admit queued graphs in arrival order while a slot and a node range are free
  while (s->qhead < s->queue.size()) {
    int slot = -1;
    for (int g = 0; g < s->gcap; ++g)
      if (!s->active[g]) { slot = g; break; }
    if (slot < 0) break;
    cldiam_server::Pending &p = s->queue[s->qhead];
    int64_t off = 0;
    if (!take_range(s, p.d.n, &off)) break;
    p.d.off = off;
    s->desc[slot] = p.d;
    s->tag[slot] = p.tag;
    s->active[slot] = 1;
    GState fresh{};
    fresh.phase = PH_START;
    CLD_HIP(hipMemcpyAsync(&s->L.desc[slot], &s->desc[slot], sizeof(GDesc), hipMemcpyHostToDevice, stream));
    CLD_HIP(hipMemcpyAsync(&job.st[slot], &fresh, sizeof(GState), hipMemcpyHostToDevice, stream));
    CLD_HIP(hipMemsetAsync(&job.cn[slot], 0, sizeof(GCount), stream));
    CLD_HIP(hipMemsetAsync(job.log + (size_t)slot * CLDIAM_STAGE_LOG * 4, 0, sizeof(int32_t) * CLDIAM_STAGE_LOG * 4,
                           stream));
    k_init_range<<<cld::blocks_for(p.d.n, 256, 4096), 256, 0, stream>>>(job, off, p.d.n);
    CLD_LAUNCH_CHECK("k_init_range");
    // the host copies above read s->desc / fresh before the next host write
    CLD_HIP(hipStreamSynchronize(stream));
    s->qhead++;
  }
  if (s->qhead > 1024 && s->qhead * 2 > s->queue.size()) {
    s->queue.erase(s->queue.begin(), s->queue.begin() + s->qhead);
    s->qhead = 0;
  }
  int nactive = 0;
  for (int g = 0; g < s->gcap; ++g) nactive += s->active[g];
  if (nactive > 0 && max_sweeps > 0) {
    CLD_HIP(hipMemsetAsync(&job.ctl->iterations, 0, sizeof(uint32_t), stream));
    for (int i = 0; i < max_sweeps; ++i) {
      launch_control(job, stream);
      k_sweep<<<s->blocks, kSweepThreads, 0, stream>>>(job);
    }
    CLD_LAUNCH_CHECK("k_sweep");
    CLD_HIP(hipMemcpyAsync(s->st_host.data(), job.st, sizeof(GState) * s->gcap, hipMemcpyDeviceToHost, stream));
    CLD_HIP(hipMemcpyAsync(s->hc, job.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    CLD_HIP(hipStreamSynchronize(stream));
    if (s->hc->error) {
      cld::set_error("server: device reported %s", cldiam_strerror(-(int)s->hc->error));
      return -(int)s->hc->error;
    }
    for (int g = 0; g < s->gcap; ++g) {
      if (!s->active[g] || s->st_host[g].phase != PH_DONE) continue;
      GCount cn;
      std::vector<int32_t> lg(CLDIAM_STAGE_LOG * 4);
      CLD_HIP(hipMemcpyAsync(&cn, &job.cn[g], sizeof cn, hipMemcpyDeviceToHost, stream));
      CLD_HIP(hipMemcpyAsync(lg.data(), job.log + (size_t)g * CLDIAM_STAGE_LOG * 4, sizeof(int32_t) * lg.size(),
                             hipMemcpyDeviceToHost, stream));
      const GState idle = [] { GState x{}; x.phase = PH_IDLE; return x; }();
      CLD_HIP(hipMemcpyAsync(&job.st[g], &idle, sizeof(GState), hipMemcpyHostToDevice, stream));
      CLD_HIP(hipStreamSynchronize(stream));
      cldiam_server::Done dn;
      dn.tag = s->tag[g];
      fill_stats(s->desc[g], s->st_host[g], cn, lg.data(), &dn.st);
      s->done.push_back(dn);
      s->active[g] = 0;
      give_range(s, s->desc[g].off, s->desc[g].n);
      --nactive;
    }
  }
  if (h_active) *h_active = nactive;
  if (h_queued) *h_queued = (int32_t)(s->queue.size() - s->qhead);
  return CLDIAM_OK;
}

extern "C" int cldiam_server_poll(cldiam_server *s, uint64_t *h_tags, cldiam_stats *h_stats, int32_t max_done,
                                  int32_t *h_ndone) {
  if (!s || !h_ndone || max_done < 0) { cld::set_error("server: invalid poll"); return CLDIAM_EINVAL; }
  int32_t k = 0;
  while (k < max_done && k < (int32_t)s->done.size()) {
    if (h_tags) h_tags[k] = s->done[k].tag;
    if (h_stats) h_stats[k] = s->done[k].st;
    ++k;
  }
  s->done.erase(s->done.begin(), s->done.begin() + k);
  *h_ndone = k;
  return CLDIAM_OK;
}
