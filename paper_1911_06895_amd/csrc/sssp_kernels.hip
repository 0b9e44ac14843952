// HIP kernels for gfx950 (CDNA4, wave64): graph validation, the light/heavy
// split of the adjacency matrix, and the persistent delta-stepping solver.
//
// The solver is one cooperative launch per call, with two 512-thread
// workgroups per compute unit (or, on request, one of 1024 threads; see Cfg).
// Every step of the method (a light phase, a heavy phase, a far-bucket
// redistribution) is processed by all workgroups; steps are
// separated by a device-wide barrier whose last arriving workgroup (the
// leader) evaluates the loop tests of Fig. 1 ("while t_Bi != 0",
// "while (t >= i*delta) != 0") and publishes the next step before releasing
// the others. Steps too small to be worth a device-wide barrier run on the
// leader workgroup alone, inside the barrier.
//
// Several sources can be solved at once: the workgroups then form groups
// (workgroup b belongs to group b % groups; with eight groups each group is one
// XCD, whose L2 keeps that group's distances). Each group has its own control
// block and working set, claims source rows from a shared counter and runs the
// schedule above over its own workgroups; the graph is shared.
//
// Memory model: every datum one workgroup writes and another reads (distances,
// stamps, lists, counters, the schedule) is written with device-scope stores
// or atomics and read with device-scope loads, which are coherent across the
// XCDs' L2 caches. The barrier therefore only needs each wave's outstanding
// stores to complete, not an L2 write-back or invalidation. Only the split
// graph (written by an earlier kernel) is read through the caches.
#include "sssp_device.h"

namespace sssp {
namespace {

// ------------------------------------------------------------------ schedule

// index of this workgroup within its group, and the group's workgroup count
__device__ inline uint32_t grp_rank(const Params& p) { return blockIdx.x / p.groups; }
__device__ inline uint32_t grp_size(const Params& p) { return gridDim.x / p.groups; }

struct Sched {
  uint32_t action, bucket, in_kind, in_count, out_buf, step, round, far_epoch, far_cur, far_base;
  uint32_t hub_parent, hub_backlog, hub_in;
  uint32_t redo;  // the current round repeats its bucket (heavy requests fell back into it; fp32)
  uint64_t lo_u, hi_u;
};

struct WgStats {
  unsigned long long light_edges, heavy_edges, improvements, attempts;
  unsigned long long step_edges, step_impr;  // since the last traced step boundary
};

// List appends of a workgroup are staged in LDS and flushed together: one
// global atomic per destination list per flush instead of one per wave.
constexpr uint32_t kSlotFront = kRingMax;     // the current bucket's next frontier
constexpr uint32_t kSlotFar = kRingMax + 1;   // the far list
constexpr uint32_t kSlotS = kRingMax + 2;     // S, the vertices expanded in this bucket
constexpr uint32_t kSlots = kRingMax + 3;     // ring slots 0..kRingMax-1, then the three above
constexpr uint32_t kNoSlot = 0xFFu;
// A frontier-list entry is a vertex id (below 2^31), for 32-bit distances with
// this bit set when the update that queued it brought the vertex into the
// current bucket from above: its first entry in the bucket, which makes it a
// member of S.
constexpr uint32_t kFreshBit = 0x80000000u;

template <uint32_t N>
struct Stage {
  uint32_t v[N];
  uint32_t rank[N];
  uint8_t slot[N];
  uint32_t n;
  uint32_t cnt[kSlots];
  uint32_t base[kSlots];
};

// Candidates that passed the prefilter (see relax_batch), queued in LDS.
template <uint32_t N>
struct Queue {
  uint32_t v[N];
  uint64_t c[N];  // candidate distance bits
  uint32_t n;     // may pass N: the excess was relaxed directly
};

// Solver configuration: the weight arithmetic plus the workgroup size. The
// default is 512-thread workgroups, two per CU, whose independent schedules
// overlap each other's latency-bound steps (faster on every workload measured);
// 1024-thread workgroups, one per CU, can be requested for one source or one
// multi-source row. Chain: the leader chains its light steps (light_chain), a
// kernel of its own so that the other kernels' code is not changed by it.
template <class Wt, uint32_t WG, bool Chain = false>
struct Cfg : Wt {
  static constexpr uint32_t kWG = WG;
  static constexpr bool kChain = Chain;
  static constexpr uint32_t kPiece = WG * kILP;  // edges of one hub piece (one round of a workgroup)
  static constexpr uint32_t kQueue = WG;         // LDS candidates (one per thread); drained once a quarter full
  // LDS staging for list appends: room for a round and a drain above the flush threshold
  static constexpr uint32_t kStage = WG * kILP + kQueue + 2048;
};

// The workgroup's state, in LDS: its group's parameters (copied from the
// launch argument at kernel start), the current schedule, the append staging,
// the candidate queue, the work counters and its view of the barrier. Device
// functions reach it through lds<W>(), which names one static LDS object per
// configuration, never through a reference parameter: the accesses then
// compile to LDS instructions (through a reference, a function that is not
// inlined would use flat ones, which wait on the global-memory counter as
// well), and the parameters are not reloaded after every global store.
template <class W>
__device__ __attribute__((always_inline)) inline Params& lds_params() {
  __shared__ Params x;
  return x;
}
template <class W>
__device__ __attribute__((always_inline)) inline Sched& lds_sched() {
  __shared__ Sched x;
  return x;
}
template <class W>
__device__ __attribute__((always_inline)) inline Stage<W::kStage>& lds_stage() {
  __shared__ Stage<W::kStage> x;
  return x;
}
template <class W>
__device__ __attribute__((always_inline)) inline WgStats& lds_stats() {
  __shared__ WgStats x;
  return x;
}
template <class W>
__device__ __attribute__((always_inline)) inline BarrierState& lds_barrier() {
  __shared__ BarrierState x;
  return x;
}
template <class W>
__device__ __attribute__((always_inline)) inline Queue<W::kQueue>& lds_queue() {
  __shared__ Queue<W::kQueue> x;
  return x;
}

// The frontier of the leader's chained light steps (see light_chain).
struct ChainList {
  uint32_t v[kChunk];
  uint32_t n;  // may pass kChunk: the excess went to the global list
};
template <class W>
__device__ __attribute__((always_inline)) inline ChainList& lds_chain() {
  __shared__ ChainList x;
  return x;
}

template <class W>
struct Lds {
  Params& p;
  Sched& s;
  Stage<W::kStage>& sg;
  WgStats& st;
  BarrierState& bar;
  Queue<W::kQueue>& q;
};

template <class W>
__device__ __attribute__((always_inline)) inline Lds<W> lds() {
  return Lds<W>{lds_params<W>(), lds_sched<W>(), lds_stage<W>(), lds_stats<W>(), lds_barrier<W>(), lds_queue<W>()};
}

// The group's record of each vertex's distance at its last light expansion in
// the current row (kInf: not expanded yet); typed like the distances.
template <class W>
__device__ __attribute__((always_inline)) inline typename W::T* texp(const Params& p) {
  return static_cast<typename W::T*>(p.texp);
}

__device__ inline void count_add(unsigned long long* field, unsigned long long v) {
  if (v) atomicAdd(field, v);
}

// i*delta <= x < (i+1)*delta for the current bucket i
template <class W>
__device__ inline bool in_bucket(typename W::T x, const Sched& s, const Params& p) {
  if constexpr (W::kInteger) return x >= s.lo_u && x < s.hi_u;
  else return W::bucket(x, p) == s.bucket;
}

// x lies above the current bucket i ((i+1)*delta <= x), or is unreachable
template <class W>
__device__ inline bool above_bucket(typename W::T x, const Sched& s, const Params& p) {
  if (x == W::kInf) return true;
  if constexpr (W::kInteger) return x >= s.hi_u;
  else return W::bucket(x, p) > s.bucket;
}

// Every workgroup's copy of the schedule the leader published. The loads are
// independent and issued together (one round trip to the coherent level).
template <class W>
__device__ inline void load_sched(Ctl* c) {
  const Lds<W> L = lds<W>();
  Sched* s = &L.s;
  if (threadIdx.x == 0) {
    const uint32_t action = ld_agent(&c->action), bucket = ld_agent(&c->bucket), in_kind = ld_agent(&c->in_kind),
                   in_count = ld_agent(&c->in_count), out_buf = ld_agent(&c->out_buf), step = ld_agent(&c->step),
                   round = ld_agent(&c->round), far_epoch = ld_agent(&c->far_epoch),
                   far_cur = ld_agent(&c->far_cur), far_base = ld_agent(&c->far_base),
                   hub_parent = ld_agent(&c->hub_parent), hub_backlog = ld_agent(&c->hub_backlog),
                   hub_in = ld_agent(&c->hub_in), redo = ld_agent(&c->redo);
    const uint64_t lo_u = ld_agent(&c->lo_u), hi_u = ld_agent(&c->hi_u);
    s->action = action;
    s->bucket = bucket;
    s->in_kind = in_kind;
    s->in_count = in_count;
    s->out_buf = out_buf;
    s->step = step;
    s->round = round;
    s->far_epoch = far_epoch;
    s->far_cur = far_cur;
    s->far_base = far_base;
    s->hub_parent = hub_parent;
    s->hub_backlog = hub_backlog;
    s->hub_in = hub_in;
    s->redo = redo;
    s->lo_u = lo_u;
    s->hi_u = hi_u;
  }
  __syncthreads();
}

// The leader publishes a new schedule (stores only; drained before the release).
__device__ inline void publish_sched(Ctl* c, const Sched& s) {
  st_agent(&c->action, s.action);
  st_agent(&c->bucket, s.bucket);
  st_agent(&c->in_kind, s.in_kind);
  st_agent(&c->in_count, s.in_count);
  st_agent(&c->out_buf, s.out_buf);
  st_agent(&c->far_base, s.far_base);
  st_agent(&c->step, s.step);
  st_agent(&c->round, s.round);
  st_agent(&c->far_epoch, s.far_epoch);
  st_agent(&c->far_cur, s.far_cur);
  st_agent(&c->hub_parent, s.hub_parent);
  st_agent(&c->hub_backlog, s.hub_backlog);
  st_agent(&c->hub_in, s.hub_in);
  st_agent(&c->redo, s.redo);
  st_agent(&c->lo_u, s.lo_u);
  st_agent(&c->hi_u, s.hi_u);
}

// Counters the leader's decision reads after a step, loaded together: the
// ring slots by the lanes of wave 0, the rest by lanes of wave 1.
enum : uint32_t { kCHubs, kCF0, kCF1, kCS, kCFar0, kCFar1, kCFarMin, kCFarMinNext, kCOvf, kCounters };
struct Counters {
  uint32_t bins[kRingMax];
  uint32_t w[kCounters];
};

__device__ inline void load_counters(Ctl* c, Counters* k) {
  const uint32_t t = threadIdx.x;
  if (t < kRingMax) {
    k->bins[t] = ld_agent(&c->bincount[t][0]);
  } else if (t >= 64 && t < 64 + kCounters) {
    const uint32_t j = t - 64;
    const uint32_t* src = j == kCHubs        ? &c->hub_count
                          : j == kCF0        ? &c->fcount[0]
                          : j == kCF1        ? &c->fcount[1]
                          : j == kCS         ? &c->scount
                          : j == kCFar0      ? &c->farcount[0]
                          : j == kCFar1      ? &c->farcount[1]
                          : j == kCFarMin    ? &c->far_min
                          : j == kCFarMinNext ? &c->far_min_next
                                             : &c->ovf_seen;
    k->w[j] = ld_agent(src);
  }
  __syncthreads();
}

// the input list of a light or heavy phase
__device__ inline const uint32_t* phase_list(const Params& p, const Sched& s, bool light) {
  if (!light) return p.slist;
  if (s.in_kind == kInBin) return p.bins + static_cast<size_t>(s.bucket & p.ring_mask) * p.n;
  return p.front[s.in_kind];
}

// ------------------------------------------------------------------ relaxation

// Traced runs only: add this workgroup's counts of the finished step to the
// control block (one atomic per workgroup), for the next trace record.
template <class W>
__device__ inline void trace_step_counts(Ctl* c) {
  const Lds<W> L = lds<W>();
  if (!L.bar.trace) return;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long te = L.st.step_edges, ti = L.st.step_impr;
    L.st.step_edges = L.st.step_impr = 0;
    if (te) g_add(&c->tr_edges, te);
    if (ti) g_add(&c->tr_impr, ti);
  }
  __syncthreads();
}

// Append winners to the ring slot of their bucket. Lanes are grouped by
// bucket with ballots only; then every group leader issues its atomic at the
// same time, so a wave waits for one atomic round trip whatever the number of
// distinct buckets.
template <class W>
__device__ inline void push_ring(bool pred, uint32_t j, uint32_t v) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  uint64_t rest = __ballot(pred);
  if (rest == 0) return;
  uint32_t my_leader = 0;
  uint64_t my_group = 0;
  while (rest) {
    const int l = first_lane(rest);
    const uint32_t jl = __builtin_amdgcn_readlane(j, l);
    const bool same = pred && j == jl;
    const uint64_t grp = __ballot(same);
    if (same) {
      my_leader = static_cast<uint32_t>(l);
      my_group = grp;
    }
    rest &= ~grp;
  }
  uint32_t base = 0;
  if (pred && lane() == my_leader)
    base = g_add(&p.ctl->bincount[j & p.ring_mask][0], static_cast<uint32_t>(__popcll(my_group)));
  base = __shfl(base, static_cast<int>(my_leader));
  if (pred) st_agent(&p.bins[static_cast<size_t>(j & p.ring_mask) * p.n + base + lanes_below(my_group)], v);
}

template <class W>
__device__ inline void stage_push(bool push, uint32_t slot, uint32_t v) {
  const Lds<W> L = lds<W>();
  auto& sg = L.sg;
  const uint64_t mask = __ballot(push);
  if (mask == 0) return;
  const int leader = first_lane(mask);
  uint32_t b = 0;
  if (static_cast<int>(lane()) == leader) b = atomicAdd(&sg.n, static_cast<uint32_t>(__popcll(mask)));
  b = __shfl(b, leader);
  if (push) {
    const uint32_t i = b + lanes_below(mask);
    sg.v[i] = v;
    sg.slot[i] = static_cast<uint8_t>(slot);
  }
}

// Move the n staged appends to their lists. All threads of the workgroup call
// it with the same n (read between two barriers, so no append raced the read).
template <class W>
__device__ void stage_flush_now(uint32_t n) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  const Sched& s = L.s;
  auto& sg = L.sg;
  if (threadIdx.x < kSlots) sg.cnt[threadIdx.x] = 0;
  __syncthreads();
  // rank of each entry within its destination: lanes grouped by destination, one LDS atomic per group
  for (uint32_t i0 = 0; i0 < n; i0 += W::kWG) {
    const uint32_t i = i0 + threadIdx.x;
    const bool valid = i < n;
    const uint32_t slot = valid ? sg.slot[i] : kNoSlot;
    uint64_t rest = __ballot(valid);
    uint32_t my_leader = 0;
    uint64_t my_group = 0;
    while (rest) {
      const int l = first_lane(rest);
      const uint32_t sl = __builtin_amdgcn_readlane(slot, l);
      const bool same = valid && slot == sl;
      const uint64_t grp = __ballot(same);
      if (same) {
        my_leader = static_cast<uint32_t>(l);
        my_group = grp;
      }
      rest &= ~grp;
    }
    uint32_t b = 0;
    if (valid && lane() == my_leader) b = atomicAdd(&sg.cnt[slot], static_cast<uint32_t>(__popcll(my_group)));
    b = __shfl(b, static_cast<int>(my_leader));
    if (valid) sg.rank[i] = b + lanes_below(my_group);
  }
  __syncthreads();
  if (threadIdx.x < kSlots) {
    const uint32_t k = threadIdx.x;
    const uint32_t c = sg.cnt[k];
    uint32_t* ctr = k < kRingMax      ? &p.ctl->bincount[k][0]
                    : k == kSlotFront ? &p.ctl->fcount[s.out_buf]
                    : k == kSlotFar   ? &p.ctl->farcount[s.far_cur]
                                      : &p.ctl->scount;
    sg.base[k] = c ? g_add(ctr, c) : 0u;
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += W::kWG) {
    const uint32_t slot = sg.slot[i];
    uint32_t* list = slot < kRingMax      ? p.bins + static_cast<size_t>(slot) * p.n
                     : slot == kSlotFront ? p.front[s.out_buf]
                     : slot == kSlotFar   ? p.far[s.far_cur]
                                          : p.slist;
    st_agent(&list[sg.base[slot] + sg.rank[i]], sg.v[i]);
  }
  __syncthreads();
  if (threadIdx.x == 0) sg.n = 0;
  __syncthreads();
}

// Chained leader steps: append a re-inserted vertex to the LDS frontier;
// returns true when it was kept there (false: it did not fit, and goes to the
// global list instead).
template <class W>
__device__ inline bool chain_push(bool push, uint32_t v) {
  ChainList& ch = lds_chain<W>();
  const uint64_t mask = __ballot(push);
  if (mask == 0) return false;
  const int leader = first_lane(mask);
  uint32_t b = 0;
  if (static_cast<int>(lane()) == leader) b = atomicAdd(&ch.n, static_cast<uint32_t>(__popcll(mask)));
  b = __shfl(b, leader);
  if (!push) return false;
  const uint32_t i = b + lanes_below(mask);
  if (i >= kChunk) return false;
  ch.v[i] = v;
  return true;
}

// A relaxation of (v, t(u) (+) w): t(v) = min(t(v), request) (Sec. III-C relax;
// Sec. IV-C/IV-D t = min(t, t_Req)), then v is filed by the bucket of its new
// tentative distance: back into the current bucket's frontier (the
// re-insertion mask (i*delta <= t_Req < (i+1)*delta) o (t_Req < t) of
// Sec. IV-C), into the ring of near buckets, or into the far list.
//
// It runs in two parts. The prefilter compares each request with a cached
// (possibly stale, never lower) copy of t(v); most requests end there. Those
// that pass are queued in LDS, and the queue is drained in bulk by the whole
// workgroup: the atomic min on t(v) and the filing, whose round trips are
// then shared by many requests instead of stalling every round.

// The atomic part for kILP candidates per lane (their atomics overlap in flight).
// kChain: the leader's chained light steps keep the re-inserted vertices in LDS.
template <class W, bool kChain = false>
__device__ inline void relax_candidates(uint64_t* t, const bool (&active)[kILP],
                                        const typename W::T (&cand)[kILP], const uint32_t (&v)[kILP],
                                        uint64_t near_end) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  const Sched& s = L.s;
  bool win[kILP];
  uint32_t jj[kILP];
  uint64_t old[kILP];
  if constexpr (W::kPacked) {
    // the word carries the frontier tag: one atomic decides the update and the re-insertion
#pragma unroll
    for (uint32_t q = 0; q < kILP; ++q) jj[q] = active[q] ? W::bucket(cand[q], p) : kNone;
#pragma unroll
    for (uint32_t q = 0; q < kILP; ++q) {
      const uint32_t tag = jj[q] <= s.bucket ? queued_tag(s.step + 1u) : 0u;
      old[q] = active[q] ? g_min(&t[v[q]], dist_word<W>(cand[q], tag)) : 0ull;
    }
#pragma unroll
    for (uint32_t q = 0; q < kILP; ++q) win[q] = active[q] && cand[q] < word_dist<W>(old[q]);
  } else {
#pragma unroll
    for (uint32_t q = 0; q < kILP; ++q) old[q] = active[q] ? g_min(&t[v[q]], cand[q]) : 0ull;
#pragma unroll
    for (uint32_t q = 0; q < kILP; ++q) win[q] = active[q] && cand[q] < old[q];
#pragma unroll
    for (uint32_t q = 0; q < kILP; ++q) jj[q] = win[q] ? W::bucket(cand[q], p) : kNone;
  }
  uint32_t slot[kILP], entry[kILP];
#pragma unroll
  for (uint32_t q = 0; q < kILP; ++q) {
    slot[q] = kNoSlot;
    entry[q] = v[q];
    if (win[q]) {
      const uint32_t j = jj[q];
      if (j <= s.bucket) {
        bool first;
        if constexpr (W::kPacked) first = tag_step(static_cast<uint32_t>(old[q])) != s.step + 1u;
        else first = g_exch(&p.qstamp[v[q]], s.step + 1u) != s.step + 1u;
        if (first) {
          slot[q] = kSlotFront;
          // (32-bit distances: the update and the re-insertion test are one atomic, so the entry
          // that makes the re-insertion is the one whose update saw the vertex above the bucket)
          if constexpr (W::kPacked)
            if (above_bucket<W>(word_dist<W>(old[q]), s, p)) entry[q] |= kFreshBit;
        }
      } else if (j < near_end) {
        // filed under bucket j unless its previous distance was in bucket j already (every
        // distance in a ring bucket came with a filing there); the stamp only tells the far
        // redistribution that the vertex has reached the ring
        const typename W::T od = word_dist<W>(old[q]);
        if (od == W::kInf || W::bucket(od, p) > j) {
          slot[q] = j & p.ring_mask;
          st_agent(&p.bstamp[v[q]], j);
        }
      } else {
        g_min(&p.ctl->far_min, j);
        if (g_exch(&p.fstamp[v[q]], s.far_epoch) != s.far_epoch) slot[q] = kSlotFar;
      }
    }
  }
  uint32_t nwin = 0, natt = 0;
#pragma unroll
  for (uint32_t q = 0; q < kILP; ++q) {
    nwin += static_cast<uint32_t>(__popcll(__ballot(win[q])));
    natt += static_cast<uint32_t>(__popcll(__ballot(active[q])));
    bool kept = false;
    if constexpr (kChain) kept = chain_push<W>(slot[q] == kSlotFront, entry[q]);
    stage_push<W>(slot[q] != kNoSlot && !kept, slot[q], entry[q]);
  }
  if (lane() == 0) {
    count_add(&L.st.improvements, nwin);
    count_add(&L.st.attempts, natt);
    count_add(&L.st.step_impr, nwin);
  }
}

// Queue the lanes' candidates; returns true for a candidate that found the
// queue full (the caller relaxes it at once).
template <class W>
__device__ inline bool queue_push(bool pass, uint32_t v, uint64_t c) {
  const Lds<W> L = lds<W>();
  const uint64_t mask = __ballot(pass);
  if (mask == 0) return false;
  const int leader = first_lane(mask);
  uint32_t b = 0;
  if (static_cast<int>(lane()) == leader) b = atomicAdd(&L.q.n, static_cast<uint32_t>(__popcll(mask)));
  b = __shfl(b, leader);
  if (!pass) return false;
  const uint32_t i = b + lanes_below(mask);
  if (i >= W::kQueue) return true;
  L.q.v[i] = v;
  L.q.c[i] = c;
  return false;
}

// The prefilter for kILP requests (v, t(u) (+) w) per lane.
template <class W, bool kChain = false>
__device__ inline void relax_batch(uint64_t* t, const bool (&active)[kILP], const typename W::T (&tu)[kILP],
                                   const uint32_t (&v)[kILP], const typename W::Wt (&w)[kILP], uint64_t near_end) {
  const Lds<W> L = lds<W>();
  using T = typename W::T;
  const Params& p = L.p;
  T cand[kILP], tv[kILP];
  bool ok[kILP];
#pragma unroll
  for (uint32_t q = 0; q < kILP; ++q) {
    ok[q] = active[q] && W::add(tu[q], w[q], &cand[q]);
    if (active[q] && !ok[q]) {
      st_agent(&p.ovf_at[v[q]], 1u);
      st_agent(&p.ctl->ovf_seen, 1u);
    }
  }
#pragma unroll
  for (uint32_t q = 0; q < kILP; ++q)
    tv[q] = ok[q] ? tload_cached<W>(t, v[q]) : T(0);  // may be stale, but never below the current value
  bool direct[kILP];
  bool any = false;
#pragma unroll
  for (uint32_t q = 0; q < kILP; ++q) {
    direct[q] = queue_push<W>(ok[q] && cand[q] < tv[q], v[q], static_cast<uint64_t>(cand[q]));
    any |= direct[q];
  }
  if (__ballot(any)) relax_candidates<W, kChain>(t, direct, cand, v, near_end);
}

// The staged-append and queue counts as every thread sees them: read between
// two barriers, so that no append or push of a faster wave races the reads.
template <class W>
__device__ inline void read_counts(uint32_t* staged, uint32_t* queued) {
  const Lds<W> L = lds<W>();
  __syncthreads();
  *staged = L.sg.n;
  *queued = L.q.n;
  __syncthreads();
}

// Flush the staged appends when another round (W::kWG * kILP appends) might not fit.
template <class W>
__device__ inline void stage_room() {
  uint32_t staged, queued;
  read_counts<W>(&staged, &queued);
  if (staged > W::kStage - W::kWG * kILP) stage_flush_now<W>(staged);
}

// Relax the `queued` candidates (read with read_counts) and empty the queue.
// All threads call it; the staging has room for W::kQueue appends.
template <class W, bool kChain = false>
__device__ void drain_queue(uint64_t* t, uint64_t near_end, uint32_t queued) {
  const Lds<W> L = lds<W>();
  using T = typename W::T;
  static_assert(W::kQueue <= W::kWG * kILP, "one pass drains the queue");
  const uint32_t n = min(queued, W::kQueue);
  for (uint32_t base = 0; base < n; base += W::kWG * kILP) {
    bool active[kILP];
    T cand[kILP];
    uint32_t v[kILP];
#pragma unroll
    for (uint32_t q = 0; q < kILP; ++q) {
      const uint32_t i = base + q * W::kWG + threadIdx.x;
      active[q] = i < n;
      v[q] = active[q] ? L.q.v[i] : 0u;
      cand[q] = active[q] ? static_cast<T>(L.q.c[i]) : T(0);
    }
    relax_candidates<W, kChain>(t, active, cand, v, near_end);
  }
  __syncthreads();
  if (threadIdx.x == 0) L.q.n = 0;
  __syncthreads();
}

// After a round of relax_batch: make room in the staging for another round,
// drain the queue once it is a quarter full (an early drain lowers t sooner,
// so fewer later requests pass the prefilter only to lose), and with `force`
// (the end of a step) drain and flush everything (a chain of the leader's
// steps keeps its appends staged until it ends).
template <class W, bool kChain = false>
__device__ inline void round_end(uint64_t* t, uint64_t near_end, bool force) {
  uint32_t staged, queued;
  read_counts<W>(&staged, &queued);
  if (staged > W::kStage - W::kWG * kILP - W::kQueue) {
    stage_flush_now<W>(staged);
    staged = 0;
  }
  if (queued >= (force ? 1u : W::kQueue / 4)) {
    drain_queue<W, kChain>(t, near_end, queued);
    if (force) read_counts<W>(&staged, &queued);
  }
  if (force && staged > 0 && !kChain) stage_flush_now<W>(staged);  // a chain defers its appends
}

// The prefilter's cached loads of t rely on every cached copy being from the
// current solve, hence stale only upward. A group's distance buffers alternate
// between its rows, so a buffer's earlier row may have left lines in this CU's
// L1 or this XCD's L2 that lie below the new row's values (the other XCDs'
// stores that reset the buffer do not reach those caches). Before the first
// step of each row, after the barrier that completes the reset, every
// workgroup therefore drops them: one agent-scope acquire invalidates both
// caches, and the workgroup barrier after it orders the other waves' loads
// behind it (one invalidation per workgroup rather than per wave).
__device__ inline void forget_cached_distances() {
  if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
}

// Work distribution over `nitems` items: in a step run by a whole group, the
// workgroup of rank b first takes item b with no atomic, then claims further
// items from a shared counter; the leader workgroup running a step alone walks
// every item in order.
__device__ inline uint32_t claim_next(uint32_t* counter, uint32_t prev, uint32_t nitems, bool solo, uint32_t size,
                                      uint32_t* s_claim) {
  if (solo) return prev + 1;
  if (nitems <= size) return nitems;  // every item was taken statically
  __syncthreads();
  if (threadIdx.x == 0) *s_claim = size + g_add(counter, 1u);
  __syncthreads();
  return *s_claim;
}

// Queue the pieces of one high-degree vertex (hub_edges or more edges in this phase).
template <class W>
__device__ inline void queue_hub(uint32_t u, uint32_t deg) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  const uint32_t pieces = (deg + W::kPiece - 1) / W::kPiece;
  uint64_t* queue = p.hub + static_cast<size_t>(1u - L.s.hub_in) * p.hub_cap;
  const uint32_t base = g_add(&p.ctl->hub_count, pieces);
  if (base + pieces > p.hub_cap) {  // cannot happen within the capacity bound; never drop work silently
    st_agent(&p.ctl->hub_full, 1u);
    st_agent(&p.ctl->abort, 1u);
  }
  for (uint32_t k = 0; k < pieces && base + k < p.hub_cap; ++k)
    st_agent(&queue[base + k], static_cast<uint64_t>(u) | (static_cast<uint64_t>(k) << 32));
}

// A group of at least this many workgroups (most of the device) hands hub
// pieces over between light phases, and by default claims chunks of at most
// kChunk / 2 entries (more chunks per workgroup: better balance over many
// workgroups) and runs steps of at most kChunk / 2 entries on the leader
// alone; smaller groups use kChunk for both. A tuning may set either limit.
constexpr uint32_t kHandOverMinGroup = 128;  // workgroups
__device__ inline uint32_t chunk_cap(const Params& p, uint32_t size) {
  if (p.chunk_entries) return p.chunk_entries;
  return size >= kHandOverMinGroup ? kChunk / 2 : kChunk;
}
__device__ inline uint32_t inline_cap(const Params& p, uint32_t size) {
  return p.inline_entries ? p.inline_entries : chunk_cap(p, size);
}

// List entries per claimed chunk: enough chunks for about four per workgroup.
// Chunk sizes are powers of two (the edge-to-entry search relies on it).
static_assert((kChunk & (kChunk - 1)) == 0 && (kMinChunk & (kMinChunk - 1)) == 0, "chunk sizes are powers of two");
__device__ inline uint32_t chunk_for(uint32_t count, uint32_t size, uint32_t cap) {
  const uint32_t target = (count + 4 * size - 1) / (4 * size);
  uint32_t c = kMinChunk;
  while (c < target && c < cap) c <<= 1;
  return c;
}

// A step run by the leader workgroup alone takes its whole list (at most
// kChunk entries) as one chunk, of the next power of two.
__device__ inline uint32_t solo_chunk(uint32_t count) {
  uint32_t c = kMinChunk;
  while (c < count && c < kChunk) c <<= 1;
  return c;
}

// Entry threadIdx.x of a step's input list, already loaded by the leader
// (steps it runs alone): the list entry, the vertex's distance word and row.
template <class T>
struct Entry {
  uint32_t u;     // as listed (with kFreshBit)
  uint64_t word;  // t(u) (with the frontier tag for 32-bit distances)
  T te;           // fp64: the distance at the vertex's last light expansion (light steps)
  uint4 row;
};

template <class W>
__device__ void hub_pieces(uint64_t* t, bool light);

// One relaxation phase: every vertex u of the input list sends t(u) (+) w along
// its light (kLight) or heavy out-edges -- the masked min-plus product
// t_Req = A_L^T (t o t_Bi) or A_H^T (t o S) of Sec. IV-C/IV-D, fused with the
// min-merge into t (the paper's fusion of the Hadamard product into vxm).
// Edges are balanced over the workgroup: the degrees of kChunk list entries
// are prefix-summed in LDS and the lanes walk the concatenated edge ranges, so
// consecutive lanes read consecutive edges of a row. Vertices with hub_edges
// or more edges are queued as pieces for a grid-wide hub step instead.
template <class W, bool kLight, bool kChain = false>
__device__ __attribute__((always_inline)) void phase(uint64_t* t, bool solo, bool preloaded = false,
                                                     Entry<typename W::T> pre = Entry<typename W::T>{}) {
  using T = typename W::T;
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  const Sched& s = L.s;
  __shared__ uint32_t s_pref[kChunk];
  __shared__ uint32_t s_beg[kChunk];
  __shared__ T s_tu[kChunk];
  __shared__ uint32_t s_wsum[W::kWG / 64];
  __shared__ uint32_t s_claim;

  const bool from_bin = kLight && s.in_kind == kInBin;
  const uint32_t* list = phase_list(p, s, kLight);
  const uint32_t count = s.in_count;
  const uint64_t near_end = static_cast<uint64_t>(s.bucket) + p.ring;  // no wrap near 2^32
  const uint32_t size = grp_size(p);
  const uint32_t chunk = solo ? solo_chunk(count) : chunk_for(count, size, chunk_cap(p, size));
  const uint32_t nchunks = (count + chunk - 1) / chunk;
  if constexpr (kLight) {
    if (!solo && s.hub_backlog > 0) hub_pieces<W>(t, true);  // the previous light phase's pieces
  }

  for (uint32_t c = solo ? 0u : grp_rank(p); c < nchunks; c = claim_next(&p.ctl->chunk_next, c, nchunks, solo, size, &s_claim)) {
    const uint32_t k = c * chunk + threadIdx.x;
    uint32_t beg = 0, deg = 0, u = 0;
    T tu = W::kInf;
    bool take = false, fresh = false;
    if (threadIdx.x < chunk && k < count) {
      const uint32_t listed = preloaded ? pre.u : ld_agent(&list[k]);
      u = listed & ~kFreshBit;
      const uint64_t word = preloaded ? pre.word : ld_agent(&t[u]);
      // the row does not depend on the distance: both loads are in flight together (a skipped
      // entry wastes its row load, one round trip less for every other)
      const uint4 row = preloaded ? pre.row : ldg(&p.rows[u]);
      tu = word_dist<W>(word);
      // a ring slot may hold vertices that have since moved to a lower bucket; a frontier vertex
      // whose light edges were already relaxed with its current distance has nothing new to send
      if constexpr (W::kPacked) {
        const uint32_t tag = static_cast<uint32_t>(word);
        take = from_bin ? in_bucket<W>(tu, s, p) : (!kLight || !tag_expanded(tag));
        fresh = kLight && !from_bin && (listed & kFreshBit) != 0u;
        // updated earlier in this step, so queued for the next one at the distance expanded
        // here: mark the word, and that entry is skipped unless a later update clears the mark
        if (kLight && take && tag == queued_tag(s.step + 1u)) (void)g_cas(&t[u], word, word & ~uint64_t(1));
      } else {
        const T te = kLight && !from_bin ? (preloaded ? pre.te : ld_agent(&texp<W>(p)[u])) : W::kInf;
        take = from_bin ? in_bucket<W>(tu, s, p) : (!kLight || tu != te);
        // fp64 updates and re-insertions are separate atomics: a vertex's first entry in the
        // bucket is recognised at its expansion instead (no expansion recorded in this row)
        fresh = kLight && !from_bin && take && te == W::kInf;
        if (kLight && take) st_agent(&texp<W>(p)[u], tu);
      }
      if (take) {
        beg = kLight ? row.x : row.y;
        deg = (kLight ? row.y : row.z) - beg;
      }
    }
    if (kLight && !p.no_heavy) {  // S = (S + t_Bi) > 0: each vertex of the bucket joins S once per round
      bool to_s = false;
      if (!s.redo) {
        // in the bucket's first round a vertex joins S once, at its first entry in the bucket:
        // its ring-slot entry (the first phase), or the entry of the update that brought it
        // into the bucket from above (distances only decrease; earlier buckets are settled)
        to_s = from_bin ? take : fresh;
      } else if (take && ld_agent(&p.sstamp[u]) != s.round) {  // a repeated round (fp32): S starts empty
        to_s = g_exch(&p.sstamp[u], s.round) != s.round;
      }
      stage_push<W>(to_s, kSlotS, u);
      stage_room<W>();
    }
    if (!solo && deg >= p.hub_edges) {
      queue_hub<W>(u, deg);
      count_add(kLight ? &L.st.light_edges : &L.st.heavy_edges, deg);
      count_add(&L.st.step_edges, deg);
      deg = 0;
    }
    uint32_t total;
    const uint32_t excl = block_exclusive_scan<W::kWG>(deg, &total, s_wsum);
    if (threadIdx.x < kChunk) {
      s_pref[threadIdx.x] = excl;
      s_beg[threadIdx.x] = beg;
      s_tu[threadIdx.x] = tu;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      count_add(kLight ? &L.st.light_edges : &L.st.heavy_edges, total);
      count_add(&L.st.step_edges, total);
    }
    const uint32_t rounds = (total + W::kWG * kILP - 1) / (W::kWG * kILP);
    for (uint32_t r = 0; r < rounds; ++r) {
      bool active[kILP];
      uint32_t v[kILP], e[kILP], at[kILP];
      typename W::Wt w[kILP];
      T tw[kILP];
#pragma unroll
      for (uint32_t q = 0; q < kILP; ++q) {
        e[q] = (r * kILP + q) * W::kWG + threadIdx.x;
        active[q] = e[q] < total;
        at[q] = 0;
      }
      // the entry owning edge e: the last one whose range starts at or before e
      // (the prefix sums do not decrease; chunk is a power of two, so every
      // search takes log2(chunk) steps and the kILP searches advance together,
      // their LDS reads in flight at once)
      if (active[0]) {  // e[0] is this lane's lowest edge
        for (uint32_t half = chunk >> 1; half > 0; half >>= 1) {
#pragma unroll
          for (uint32_t q = 0; q < kILP; ++q)
            if (s_pref[at[q] + half] <= e[q]) at[q] += half;
        }
      }
#pragma unroll
      for (uint32_t q = 0; q < kILP; ++q) {
        v[q] = 0;
        w[q] = 0;
        tw[q] = W::kInf;
        if (active[q]) {
          const uint32_t pos = s_beg[at[q]] + (e[q] - s_pref[at[q]]);
          const uint64_t ed = ldg(&p.edges[pos]);
          v[q] = static_cast<uint32_t>(ed);
          w[q] = W::weight(p, ed, pos);
          tw[q] = s_tu[at[q]];
        }
      }
      relax_batch<W, kChain>(t, active, tw, v, w, near_end);
      round_end<W, kChain>(t, near_end, false);
    }
    __syncthreads();
  }
  round_end<W, kChain>(t, near_end, true);
}

template <class W>
__device__ void light_chain(uint64_t* t, Entry<typename W::T> e);

// The leader's steps run alone (inside the barrier) call this out-of-line
// copy; the group-wide steps of the kernel's loop have the phase inlined, so
// that their workgroups do not save and restore registers around a call at
// every step. With W::kChain a light step starts a chain of them (light_chain).
template <class W, bool kLight>
__device__ __attribute__((noinline)) void phase_solo(uint64_t* t, Entry<typename W::T> pre) {
  if constexpr (kLight && W::kChain) light_chain<W>(t, pre);
  else phase<W, kLight>(t, true, true, pre);
}

// Hub pieces: W::kPiece consecutive edges of the high-degree vertices queued by
// the previous phase (light or heavy edges, per `light`), spread over all
// workgroups. They are a step of their own (a hub step), or, when the
// previous phase was a light phase whose frontier is not empty, the first
// work of the next light phase (relaxations commute, and the phase's
// re-insertions are simply found one phase later).
template <class W>
__device__ void hub_pieces(uint64_t* t, bool light) {
  const Lds<W> L = lds<W>();
  using T = typename W::T;
  const Params& p = L.p;
  const Sched& s = L.s;
  constexpr uint32_t kPerMax = 2;
  __shared__ uint32_t s_beg[kPerMax], s_end[kPerMax], s_claim;
  __shared__ T s_tu[kPerMax];
  const uint64_t* queue = p.hub + static_cast<size_t>(s.hub_in) * p.hub_cap;
  const uint32_t count = s.hub_backlog < p.hub_cap ? s.hub_backlog : p.hub_cap;
  const uint64_t near_end = static_cast<uint64_t>(s.bucket) + p.ring;  // no wrap near 2^32
  const uint32_t size = grp_size(p);
  // A claim takes two consecutive pieces when there are at least eight per
  // workgroup (their rows and distances then come in one round trip), else
  // one (the step lasts as long as its busiest workgroup). Workgroup b takes
  // claim b, then claims further ones from a counter. Thread 0 works one claim
  // ahead: while a claim is relaxed, the next one is already claimed and its
  // queue records are in flight, so a claim boundary waits only for the rows
  // and t(u) of its vertices.
  const uint32_t per = count >= 8u * size ? 2u : 1u;
  const uint32_t claims = (count + per - 1) / per;
  uint32_t c = grp_rank(p);
  uint64_t rec[kPerMax] = {0ull, 0ull};  // thread 0: queue records of claim c
  if (threadIdx.x == 0 && c < claims) {
#pragma unroll
    for (uint32_t q = 0; q < kPerMax; ++q)
      if (q < per && c * per + q < count) rec[q] = ld_agent(&queue[c * per + q]);
  }
  while (c < claims) {
    if (threadIdx.x == 0) {
      const uint32_t nc = claims <= size ? claims : size + g_add(&p.ctl->hub_next, 1u);
      uint4 row[kPerMax];
      T tu[kPerMax];
      uint32_t piece[kPerMax];
      bool valid[kPerMax];
#pragma unroll
      for (uint32_t q = 0; q < kPerMax; ++q) {
        valid[q] = q < per && c * per + q < count;
        const uint32_t u = static_cast<uint32_t>(rec[q]);
        piece[q] = static_cast<uint32_t>(rec[q] >> 32);
        if (valid[q]) {
          row[q] = ldg(&p.rows[u]);
          tu[q] = tload<W>(t, u);
        }
      }
#pragma unroll
      for (uint32_t q = 0; q < kPerMax; ++q)
        rec[q] = q < per && nc < claims && nc * per + q < count ? ld_agent(&queue[nc * per + q]) : 0ull;
#pragma unroll
      for (uint32_t q = 0; q < kPerMax; ++q) {
        s_beg[q] = s_end[q] = 0;
        if (valid[q]) {
          const uint32_t b = light ? row[q].x : row[q].y;
          const uint32_t e = light ? row[q].y : row[q].z;
          const uint32_t pb = b + piece[q] * W::kPiece;
          s_beg[q] = pb;
          s_end[q] = e - pb > W::kPiece ? pb + W::kPiece : e;
          s_tu[q] = tu[q];
        }
      }
      s_claim = nc;
    }
    __syncthreads();
    c = s_claim;
    for (uint32_t q = 0; q < per; ++q) {
      const uint32_t pbeg = s_beg[q], pend = s_end[q];
      if (pbeg >= pend) continue;  // the last claim's missing second piece
      bool active[kILP];
      uint32_t v[kILP];
      typename W::Wt w[kILP];
      T tw[kILP];
#pragma unroll
      for (uint32_t i = 0; i < kILP; ++i) {
        const uint32_t e = pbeg + i * W::kWG + threadIdx.x;
        active[i] = e < pend;
        v[i] = 0;
        w[i] = 0;
        tw[i] = s_tu[q];
        if (active[i]) {
          const uint64_t ed = ldg(&p.edges[e]);
          v[i] = static_cast<uint32_t>(ed);
          w[i] = W::weight(p, ed, e);
        }
      }
      relax_batch<W>(t, active, tw, v, w, near_end);
      round_end<W>(t, near_end, false);
    }
    __syncthreads();  // every thread has read this claim's pieces before thread 0 writes the next
  }
  round_end<W>(t, near_end, true);
}

// Far-list redistribution: far vertices whose bucket is now within the ring
// move into it; the rest move to the other far list.
template <class W>
__device__ void far_step(uint64_t* t) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  const Sched& s = L.s;
  const uint32_t count = s.in_count;
  const uint32_t* list = p.far[s.far_cur];
  const uint32_t nxt = 1u - s.far_cur;
  const uint64_t near_end = static_cast<uint64_t>(s.far_base) + p.ring;
  const uint32_t size = grp_size(p), rank = grp_rank(p);
  const uint32_t iters = (count + size * W::kWG - 1) / (size * W::kWG);
  for (uint32_t it = 0; it < iters; ++it) {
    const uint32_t k = (it * size + rank) * W::kWG + threadIdx.x;
    bool to_ring = false, to_far = false;
    uint32_t v = 0, j = 0;
    if (k < count) {
      v = ld_agent(&list[k]);
      // still only filed far (never moved into the ring since)?
      if (ld_agent(&p.bstamp[v]) == kNone) {
        j = W::bucket(tload<W>(t, v), p);
        if (j < near_end) {
          to_ring = g_min(&p.bstamp[v], j) > j;
        } else {
          g_min(&p.ctl->far_min_next, j);
          to_far = g_exch(&p.fstamp[v], s.far_epoch + 1u) != s.far_epoch + 1u;
        }
      }
    }
    push_ring<W>(to_ring, j, v);
    push_wave(p.far[nxt], &p.ctl->farcount[nxt], to_far, v);
  }
}

// A candidate that did not fit marked its target; the distance of that target
// is unrepresentable exactly when no other path reached it.
template <class W>
__device__ void overflow_step(uint64_t* t) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  for (uint32_t v = grp_rank(p) * W::kWG + threadIdx.x; v < p.n; v += grp_size(p) * W::kWG) {
    if (ld_agent(&p.ovf_at[v])) {
      if (tload<W>(t, v) == W::kInf) st_agent(&p.ctl->ovf_real, 1u);
      st_agent(&p.ovf_at[v], 0u);
    }
  }
}

// ------------------------------------------------------------------ leader decisions

// Bucket i: [i*delta, (i+1)*delta) as integer bounds (integer weights).
template <class W>
__device__ inline void set_bucket(uint32_t i) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  Sched* s = &L.s;
  s->bucket = i;
  s->lo_u = static_cast<uint64_t>(i) * p.delta_u;
  s->hi_u = static_cast<uint64_t>(i + 1ull) * p.delta_u;
}

// Next bucket to process: the first non-empty ring slot among the `len`
// buckets starting at `from`, unless far-future vertices (fc of them, none
// below bucket fmin) may come first. Wave 0 scans the slots; thread 0 decides.
template <class W>
__device__ void choose_next(const Counters& k, uint32_t from, uint32_t len, uint32_t fc, uint32_t fmin) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  Sched* s = &L.s;
  __shared__ uint32_t s_jn;
  if (threadIdx.x < 64) {
    const uint32_t l = threadIdx.x;
    const bool nonempty = l < len && k.bins[(from + l) & p.ring_mask] != 0u;
    const uint64_t m = __ballot(nonempty);
    if (l == 0) s_jn = m ? from + static_cast<uint32_t>(first_lane(m)) : kNone;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t jn = s_jn;
    if (fc > 0 && (jn == kNone || fmin <= jn)) {
      s->action = kActFar;
      s->far_base = jn == kNone ? fmin : min(jn, fmin);
      s->in_count = fc;
    } else if (jn == kNone) {
      s->action = k.w[kCOvf] ? kActOverflowCheck : kActDone;
    } else {  // B_i = {v : i*delta <= t(v) < (i+1)*delta} for the smallest non-empty i
      set_bucket<W>(jn);
      s->action = kActLight;
      s->redo = 0u;
      s->in_kind = kInBin;
      s->in_count = k.bins[jn & p.ring_mask];
      s->out_buf = 0u;
      g_add(&p.ctl->buckets, 1ull);
    }
  }
  __syncthreads();
}

// Start a solve: t = inf was set by every workgroup; t(s) = 0 for each seed
// (Fig. 1 left, initialisation; with several seeds, d(v) is the distance from
// the nearest one), and the seeds form B_0. Seeds outside [0, n) are reported
// and skipped; repeated seeds are filed once. The schedule of the first step
// is left in *s and published. `reset_tags`: the group's stamps were just
// cleared, so the de-duplication tags restart.
template <class W>
__device__ void leader_start(uint64_t* t, const int32_t* seeds, int nseeds, bool reset_tags) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  Sched* s = &L.s;
  Ctl* c = p.ctl;
  if (threadIdx.x < kRingMax) st_agent(&c->bincount[threadIdx.x][0], 0u);
  if (threadIdx.x == 0) {
    uint32_t step = 0, round = 0, far_epoch = 1;
    if (!reset_tags) {
      step = ld_agent(&c->step);
      round = ld_agent(&c->round);
      far_epoch = ld_agent(&c->far_epoch);
    }
    g_add(&c->sources, 1ull);
    st_agent(&c->fcount[0], 0u);
    st_agent(&c->fcount[1], 0u);
    st_agent(&c->scount, 0u);
    st_agent(&c->farcount[0], 0u);
    st_agent(&c->farcount[1], 0u);
    st_agent(&c->far_min, kNone);
    st_agent(&c->far_min_next, kNone);
    st_agent(&c->ovf_seen, 0u);
    st_agent(&c->hub_count, 0u);
    st_agent(&c->chunk_next, 0u);
    st_agent(&c->hub_next, 0u);
    Sched n{};
    n.step = step + 1u;
    n.round = round + 1u;
    n.far_epoch = far_epoch;
    *s = n;
  }
  drain_stores();
  __syncthreads();
  for (int i = threadIdx.x; i < nseeds; i += W::kWG) {
    const int32_t src = ldg(&seeds[i]);
    if (src < 0 || static_cast<uint32_t>(src) >= p.n) {
      st_agent(&c->bad_source, 1u);
      continue;
    }
    const uint32_t u = ldg(&p.vid[src]);
    tstore<W>(t, u, typename W::T(0));
    if (g_min(&p.bstamp[u], 0u) != 0u) st_agent(&p.bins[g_add(&c->bincount[0][0], 1u)], u);
  }
  drain_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    set_bucket<W>(0u);
    s->action = kActLight;
    s->in_kind = kInBin;
    s->in_count = ld_agent(&c->bincount[0][0]);
    s->out_buf = 0u;
    g_add(&c->buckets, 1ull);
    publish_sched(c, *s);
  }
  drain_stores();
  __syncthreads();
}

// Schedule the step that follows the completed step *s (the leader's copy in
// LDS, replaced by the new schedule, which is also published). The counters
// are read in one round trip; the rest is stores, which the caller drains
// before anything reads them back (the barrier release does).
template <class W>
__device__ void after_step() {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  Sched* s = &L.s;
  Ctl* c = p.ctl;
  __shared__ Counters k;
  __shared__ uint32_t s_next, s_fc, s_fmin;  // s_next 0: decided; 1: next bucket after s.bucket; 2: after a far step
  load_counters(c, &k);
  if (threadIdx.x == 0) {
    const Sched o = *s;
    Sched n = o;
    uint32_t next = 0;
    st_agent(&c->chunk_next, 0u);
    st_agent(&c->hub_next, 0u);
    const uint32_t hubs = k.w[kCHubs];  // pieces queued by the finished step (a hub step queues none)
    const bool phase_done = o.action == kActLight || o.action == kActHeavy;
    // A light phase that re-inserted vertices hands its pieces to the next light
    // phase (saving a barrier), in a group that spans most of the device (where
    // a barrier is dearest) and unless that phase is small enough for the
    // leader to run alone.
    const bool hand_over = o.action == kActLight && hubs > 0 && grp_size(p) >= kHandOverMinGroup &&
                           k.w[o.out_buf ? kCF1 : kCF0] > kChunk / 2;
    n.hub_backlog = 0;
    if (phase_done && hubs > 0 && !hand_over) {  // finish the phase: its high-degree vertices
      n.hub_parent = o.action;
      n.hub_backlog = hubs;
      n.hub_in = 1u - o.hub_in;
      n.action = kActHub;
    } else {
      const uint32_t parent = o.action == kActHub ? o.hub_parent : o.action;
      st_agent(&c->hub_count, 0u);
      if (hand_over) {
        n.hub_backlog = hubs;
        n.hub_in = 1u - o.hub_in;
      }
      if (parent == kActLight) {
        g_add(&c->light_phases, 1ull);
        n.step = o.step + 1u;
        const uint32_t n_next = k.w[o.out_buf ? kCF1 : kCF0];
        if (o.in_kind == kInBin) st_agent(&c->bincount[o.bucket & p.ring_mask][0], 0u);
        else st_agent(&c->fcount[o.in_kind], 0u);
        if (n_next > 0) {  // while t_Bi != 0: another light phase on the re-inserted vertices
          n.action = kActLight;
          n.in_kind = o.out_buf;
          n.in_count = n_next;
          n.out_buf = 1u - o.out_buf;
        } else if (p.no_heavy) {  // A_H is empty (every weight <= delta): the bucket is done
          next = 1;
        } else {  // B_i is empty: one heavy phase over S
          n.action = kActHeavy;
          n.in_count = k.w[kCS];
        }
      } else if (parent == kActHeavy) {
        g_add(&c->heavy_phases, 1ull);
        n.step = o.step + 1u;
        n.round = o.round + 1u;
        st_agent(&c->scount, 0u);
        // A heavy request can only fall back into bucket i through fp32 rounding
        // (t(u) + w > (i+1)*delta in exact arithmetic); such vertices restart bucket i.
        const uint32_t n_redo = k.w[o.out_buf ? kCF1 : kCF0];
        if (n_redo > 0) {
          n.action = kActLight;
          n.in_kind = o.out_buf;
          n.in_count = n_redo;
          n.out_buf = 1u - o.out_buf;
          n.redo = 1u;
        } else {
          next = 1;
        }
      } else if (parent == kActFar) {
        g_add(&c->far_phases, 1ull);
        n.step = o.step + 1u;
        st_agent(&c->farcount[o.far_cur], 0u);
        n.far_cur = 1u - o.far_cur;
        st_agent(&c->far_min, k.w[kCFarMinNext]);
        st_agent(&c->far_min_next, kNone);
        n.far_epoch = o.far_epoch + 1u;
        next = 2;
      } else {  // overflow check
        n.action = kActDone;
      }
    }
    // far lists as the next-bucket choice sees them (after a far step: the other list)
    s_fc = k.w[n.far_cur ? kCFar1 : kCFar0];
    s_fmin = next == 2 ? k.w[kCFarMinNext] : k.w[kCFarMin];
    *s = n;
    s_next = next;
  }
  __syncthreads();
  const uint32_t next = s_next;
  if (next == 1) choose_next<W>(k, s->bucket + 1u, p.ring - 1u, s_fc, s_fmin);
  else if (next == 2) choose_next<W>(k, s->far_base, p.ring, s_fc, s_fmin);
  if (threadIdx.x == 0) publish_sched(c, *s);
  __syncthreads();
}

// Edges a light or heavy step would scan (its list has at most inline_cap <= kChunk entries);
// each thread keeps its entry for the phase that may follow on this workgroup.
template <bool kLight, class W>
__device__ uint32_t step_edges(const uint64_t* t, uint32_t* s_wsum, Entry<typename W::T>* e) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  const Sched& s = L.s;
  const uint32_t* list = phase_list(p, s, kLight);
  uint32_t deg = 0;
  if (threadIdx.x < s.in_count) {
    e->u = ld_agent(&list[threadIdx.x]);
    const uint32_t u = e->u & ~kFreshBit;
    e->word = ld_agent(&t[u]);
    e->row = ldg(&p.rows[u]);
    deg = kLight ? e->row.y - e->row.x : e->row.z - e->row.y;
    if (kLight && s.in_kind != kInBin) {  // nothing new to send: the phase skips it
      if constexpr (W::kPacked) {
        if (tag_expanded(static_cast<uint32_t>(e->word))) deg = 0;
      } else {
        e->te = ld_agent(&texp<W>(p)[u]);
        if (e->word == e->te) deg = 0;
      }
    }
  }
  uint32_t total;
  (void)block_exclusive_scan<W::kWG>(deg, &total, s_wsum);
  return total;
}

// The leader's chained light steps. A light step the leader runs alone keeps
// the vertices it re-inserts in LDS; while they are few enough for another
// step of its own (the limits of the steps the leader runs alone), the next
// light phase of the bucket starts from them at once: no list append and
// read-back, no counter round trip, no schedule publication in between. The
// schedule in LDS advances as after_step would advance it, and the other
// appends (S, the ring, the far list) stay staged until the chain ends. Then
// the LDS frontier goes to the global list as the last step's output, and
// after_step takes over. Repeated rounds (fp32) run one step at a time.
constexpr uint32_t kChainMax = 4096;  // steps per chain at most
template <class W>
__device__ __attribute__((always_inline)) void light_chain(uint64_t* t, Entry<typename W::T> e) {
  using T = typename W::T;
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  Sched& s = L.s;
  ChainList& ch = lds_chain<W>();
  Ctl* c = p.ctl;
  __shared__ uint32_t s_wsum[W::kWG / 64];
  if (s.redo) {
    phase<W, true>(t, true, true, e);
    return;
  }
  for (uint32_t k = 0;; ++k) {
    if (threadIdx.x == 0) ch.n = 0;
    __syncthreads();
    phase<W, true, true>(t, true, true, e);
    __syncthreads();
    const uint32_t n = ch.n;
    bool go = false;
    if (n > 0 && n <= inline_cap(p, grp_size(p)) && k + 1 < kChainMax) {
      // the next step's entries, one per thread: vertex, distance word, row
      e = Entry<T>{};
      uint32_t deg = 0, total;
      if (threadIdx.x < n) {
        e.u = ch.v[threadIdx.x];
        const uint32_t u = e.u & ~kFreshBit;
        e.word = ld_agent(&t[u]);
        e.row = ldg(&p.rows[u]);
        deg = e.row.y - e.row.x;
        if constexpr (W::kPacked) {
          if (tag_expanded(static_cast<uint32_t>(e.word))) deg = 0;  // nothing new to send
        } else {
          e.te = ld_agent(&texp<W>(p)[u]);
          if (e.word == e.te) deg = 0;
        }
      }
      (void)block_exclusive_scan<W::kWG>(deg, &total, s_wsum);
      go = total <= p.inline_edges;
    }
    if (!go) {  // the LDS frontier becomes the last step's output list
      stage_room<W>();
      const uint32_t kept = min(n, kChunk);
      stage_push<W>(threadIdx.x < kept, kSlotFront, threadIdx.x < kept ? ch.v[threadIdx.x] : 0u);
      uint32_t staged, queued;
      read_counts<W>(&staged, &queued);
      if (staged > 0) stage_flush_now<W>(staged);
      return;
    }
    // the schedule of the next step, as after_step would set it
    trace_step_counts<W>(c);
    if (threadIdx.x == 0) {
      g_add(&c->light_phases, 1ull);
      if (k == 0) {  // the first step's input was a global list, now consumed
        if (s.in_kind == kInBin) st_agent(&c->bincount[s.bucket & p.ring_mask][0], 0u);
        else st_agent(&c->fcount[s.in_kind], 0u);
      }
      s.step += 1u;
      s.in_kind = s.out_buf;
      s.in_count = n;
      s.out_buf = 1u - s.out_buf;
      if (L.bar.trace) publish_sched(c, s);
      g_add(&c->heartbeat, 1u);  // the waiting workgroups see progress
    }
    // the count reset lands before any later append to that list; fp64: the expansion
    // records are read back by the next step
    if (k == 0 || L.bar.trace || !W::kPacked) drain_stores();
    __syncthreads();
    if (threadIdx.x == 0) record_trace(c, L.bar.trace, 0x80u);
  }
}

// The leader's part of a barrier: schedule the step after `s`; while that step
// is a small light or heavy phase, run it on this workgroup alone and schedule again.
template <class W>
__device__ void lead(uint64_t* t, bool schedule_first) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  Sched* s = &L.s;
  __shared__ uint32_t s_wsum[W::kWG / 64];
  if (schedule_first) after_step<W>();
  for (;;) {  // *s is the current schedule (set by leader_start or after_step)
    const bool light = s->action == kActLight;
    if (!(light || s->action == kActHeavy) || s->in_count > inline_cap(p, grp_size(p)) || s->hub_backlog > 0) break;
    Entry<typename W::T> e{};
    const uint32_t edges = light ? step_edges<true, W>(t, s_wsum, &e) : step_edges<false, W>(t, s_wsum, &e);
    if (edges > p.inline_edges) break;
    drain_stores();  // the counter resets of after_step land before this step's appends
    __syncthreads();
    if (threadIdx.x == 0) record_trace(p.ctl, L.bar.trace, 0x80u);
    if (threadIdx.x == 0) g_add(&p.ctl->heartbeat, 1u);  // the waiting workgroups see progress
    if (light) phase_solo<W, true>(t, e);
    else phase_solo<W, false>(t, e);
    trace_step_counts<W>(p.ctl);
    drain_stores();
    __syncthreads();
    after_step<W>();
  }
}

// The leader's part of the barrier that starts a solve: claim the next row of
// the batch and initialise its solve, or mark the group finished. A row is one
// source, or (multi) all k sources at once in a single row.
template <class W>
__device__ void leader_claim(uint64_t* t, const int32_t* sources, int k, int multi, bool reset_tags) {
  const Lds<W> L = lds<W>();
  const Params& p = L.p;
  __shared__ uint32_t s_row;
  Ctl* c = p.ctl;
  if (threadIdx.x == 0) {
    const uint32_t r = g_add(p.next_source, 1u);
    const uint32_t rows = multi ? 1u : static_cast<uint32_t>(k);
    s_row = r < rows ? r : kNone;
    st_agent(&c->source_index, s_row);
  }
  __syncthreads();
  const uint32_t r = s_row;
  if (r == kNone) return;
  forget_cached_distances();  // the inline steps below use the prefilter
  leader_start<W>(t, multi ? sources : sources + r, multi ? k : 1, reset_tags);
  lead<W>(t, false);  // the first phases (around the seeds) are usually small
}

template <class W>
__global__ __launch_bounds__(W::kWG, 4) void solver_kernel(const Params* __restrict__ params, uint32_t groups,
                                                     const int32_t* sources, int k, int multi, void* dist) {
  const Lds<W> L = lds<W>();
  using T = typename W::T;
  __shared__ uint32_t s_row;
  if (threadIdx.x == 0) {
    L.p = params[blockIdx.x % groups];
    L.sg.n = 0;
    L.q.n = 0;
    L.st = WgStats{0, 0, 0, 0, 0, 0};
  }
  __syncthreads();
  const Params& p = L.p;
  const uint32_t rank = grp_rank(p), size = grp_size(p);
  Ctl* c = p.ctl;
  init_barrier(c, L.bar);
  bool alive = true;
  for (uint32_t it = 0; alive; ++it) {
    // the de-duplication tags grow by one per step and per bucket: long before
    // they could wrap, the group clears its stamps and restarts the tags (every
    // workgroup reads the same tags: the leader changes them only after this
    // barrier's arrival)
    const bool reset_tags = ld_agent(&c->step) > kEpochLimit || ld_agent(&c->round) > kEpochLimit ||
                            ld_agent(&c->far_epoch) > kEpochLimit;
    // distances live in solver ids; a group's consecutive sources alternate
    // buffers so that copying out one row never races with initialising the next
    uint64_t* t = static_cast<uint64_t*>(p.tbuf[it & 1]);
    for (uint32_t v = rank * W::kWG + threadIdx.x; v < p.n; v += size * W::kWG) {
      tstore<W>(t, v, W::kInf);
      if constexpr (!W::kPacked) st_agent(&texp<W>(p)[v], W::kInf);
      st_agent(&p.bstamp[v], kNone);
      if (reset_tags) {
        st_agent(&p.qstamp[v], 0u);
        st_agent(&p.sstamp[v], 0u);
        st_agent(&p.fstamp[v], 0u);
      }
    }
    alive = grid_sync(c, size, rank, L.bar, [&] { leader_claim<W>(t, sources, k, multi, reset_tags); });
    if (threadIdx.x == 0) s_row = ld_agent(&c->source_index);
    __syncthreads();
    const uint32_t row = s_row;
    if (!alive || row == kNone) break;
    forget_cached_distances();
    while (alive) {
      load_sched<W>(c);
      const uint32_t a = L.s.action;
      if (a == kActDone) break;
      if (a == kActLight) phase<W, true>(t, false);
      else if (a == kActHeavy) phase<W, false>(t, false);
      else if (a == kActHub) hub_pieces<W>(t, L.s.hub_parent == kActLight);
      else if (a == kActFar) far_step<W>(t);
      else if (a == kActOverflowCheck) overflow_step<W>(t);
      else if (threadIdx.x == 0) st_agent(&c->abort, 1u);
      trace_step_counts<W>(c);
      alive = grid_sync(c, size, rank, L.bar, [&] { lead<W>(t, true); });
    }
    if (alive) {  // the source's row of the output, in the caller's vertex numbering
      T* out = static_cast<T*>(dist) + static_cast<size_t>(row) * p.n;
      // a vertex without in-edges is reached only as a seed: a one-source row gives the others
      // infinity without reading t (about half the vertices of an R-MAT graph); four vertices per
      // thread are read before any is written, so their round trips overlap
      const uint32_t src = multi ? kNone : static_cast<uint32_t>(ldg(&sources[row]));
      const uint32_t zf = multi ? p.n : p.zero_from;
      const uint32_t stride = size * W::kWG;
      uint32_t v = rank * W::kWG + threadIdx.x;
      for (; v + 3u * stride < p.n; v += 4u * stride) {
        uint32_t id[4];
        T d[4];
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) id[q] = ldg(&p.vid[v + q * stride]);
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) d[q] = id[q] < zf || v + q * stride == src ? tload<W>(t, id[q]) : W::kInf;
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) *gp(&out[v + q * stride]) = d[q];
      }
      for (; v < p.n; v += stride) {
        const uint32_t id = ldg(&p.vid[v]);
        *gp(&out[v]) = id < zf || v == src ? tload<W>(t, id) : W::kInf;
      }
    }
  }
  // add this workgroup's counters to the group's control block
  __syncthreads();
  if (threadIdx.x == 0) {
    if (L.st.light_edges) g_add(&c->light_edges, L.st.light_edges);
    if (L.st.heavy_edges) g_add(&c->heavy_edges, L.st.heavy_edges);
    if (L.st.improvements) g_add(&c->improvements, L.st.improvements);
    if (L.st.attempts) g_add(&c->attempts, L.st.attempts);
  }
}

// Prepare the control blocks of `groups` groups for a launch: clear the
// counters, the abort flag and the batch's source counter (and the tags when
// the de-duplication stamps were just cleared). Only the first group traces.
__global__ void ctl_reset_kernel(Ctl* ctls, uint32_t groups, int reset_epochs, unsigned long long* trace,
                                 uint32_t trace_cap, unsigned long long wait_ticks) {
  const uint32_t g = threadIdx.x;
  if (g >= groups) return;
  Ctl* c = ctls + g;
  c->trace = g == 0 ? trace : nullptr;
  c->trace_cap = g == 0 ? trace_cap : 0u;
  c->trace_len = 0;
  c->tr_edges = 0;
  c->tr_impr = 0;
  for (uint32_t b = 0; b < kBarGroups; ++b) c->bar_sub[b][0] = 0;
  c->bar_arrive = 0;
  c->abort = 0;
  c->ovf_real = 0;
  c->next_source = 0;
  c->bad_source = 0;
  c->hub_full = 0;
  c->wait_ticks = wait_ticks;
  c->source_index = kNone;
  c->sources = c->buckets = c->light_phases = c->heavy_phases = c->far_phases = 0;
  c->light_edges = c->heavy_edges = c->improvements = c->attempts = c->barriers = 0;
  c->adj_released = 0;
  if (reset_epochs) {
    c->step = 0;
    c->round = 0;
    c->far_epoch = 1;  // stamps are zero: every tag starts above 0
  }
}

__global__ void fill_kernel(uint32_t* p, size_t count, uint32_t value) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = value;
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_ctl_reset(Ctl* c, uint32_t groups, int reset_epochs, unsigned long long* trace, uint32_t trace_cap,
                            unsigned long long wait_ticks, hipStream_t s) {
  if (groups < 1 || groups > kMaxGroups) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ctl_reset_kernel, dim3(1), dim3(kMaxGroups), 0, s, c, groups, reset_epochs, trace, trace_cap,
                     wait_ticks);
  return hipGetLastError();
}

hipError_t launch_fill(uint32_t* p, size_t count, uint32_t value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + kAuxWG - 1) / kAuxWG;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(kAuxWG), 0, s, p, count, value);
  return hipGetLastError();
}

namespace {
// the solver kernel of a weight type, workgroup size and step chaining
template <uint32_t WG, bool Chain>
const void* solver_fn(uint32_t wtype) {
  return wtype == kWU32   ? reinterpret_cast<const void*>(solver_kernel<Cfg<WeightU32, WG, Chain>>)
         : wtype == kWF32 ? reinterpret_cast<const void*>(solver_kernel<Cfg<WeightF32, WG, Chain>>)
                          : reinterpret_cast<const void*>(solver_kernel<Cfg<WeightF64, WG, Chain>>);
}
const void* solver_fn(uint32_t wtype, int wg, bool chain) {
  if (wg == kWGGroups) return chain ? solver_fn<kWGGroups, true>(wtype) : solver_fn<kWGGroups, false>(wtype);
  return chain ? solver_fn<kWG, true>(wtype) : solver_fn<kWG, false>(wtype);
}
}  // namespace

hipError_t solver_occupancy(int wtype, int wg, bool chain, int* blocks_per_cu) {
  if (wg != kWG && wg != kWGGroups) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, solver_fn(static_cast<uint32_t>(wtype), wg, chain),
                                                      wg, 0);
}

// One cooperative launch (every workgroup co-resident, which the barriers
// need). While the stream is being captured into a graph, the launch-attribute
// form records a cooperative kernel node.
hipError_t launch_solver(const Params* params, uint32_t groups, uint32_t wtype, const int32_t* sources, int k,
                         int multi, void* dist, int grid, int wg, bool chain, hipStream_t s) {
  if (groups < 1 || groups > kMaxGroups || grid < 1 || grid % static_cast<int>(groups) != 0) return hipErrorInvalidValue;
  if (wg != kWG && wg != kWGGroups) return hipErrorInvalidValue;
  const Params* pp = params;
  uint32_t gg = groups;
  const int32_t* src = sources;
  int kk = k;
  int mm = multi;
  void* d = dist;
  void* args[] = {&pp, &gg, &src, &kk, &mm, &d};
  const void* fn = solver_fn(wtype, wg, chain);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(s, &cap);
  if (e != hipSuccess) return e;
  if (cap == hipStreamCaptureStatusNone) return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(wg), args, 0, s);
  hipLaunchAttribute attr[1] = {};
  attr[0].id = hipLaunchAttributeCooperative;
  attr[0].val.cooperative = 1;
  hipLaunchConfig_t cfg{};
  cfg.gridDim = dim3(static_cast<uint32_t>(grid));
  cfg.blockDim = dim3(static_cast<uint32_t>(wg));
  cfg.dynamicSmemBytes = 0;
  cfg.stream = s;
  cfg.attrs = attr;
  cfg.numAttrs = 1;
  return hipLaunchKernelExC(&cfg, fn, args);
}

}  // namespace sssp
