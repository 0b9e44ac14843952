// Device helpers shared by the solver and the adjoint: device-scope loads and
// stores, wave-level utilities, the weight arithmetic and the grid barrier.
#pragma once

#include "sssp_internal.h"

namespace sssp {
namespace {

// ------------------------------------------------------------------ helpers

// Every pointer the kernels dereference here points to device (global) memory:
// accesses through these views compile to global_* instructions rather than
// flat ones (no LDS-aperture check, and no LDS wait counter to drain).
template <typename T>
__device__ inline __attribute__((address_space(1))) T* gp(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ inline const __attribute__((address_space(1))) T* gp(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// plain (cached) load
template <typename T>
__device__ inline T ldg(const T* p) {
  return *gp(p);
}

__device__ inline uint4 ldg(const uint4* p) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const v4u v = *(const __attribute__((address_space(1))) v4u*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}

// device-scope (coherent across the XCDs) load, store and atomics
template <typename T>
__device__ inline T ld_agent(const T* p) {
  return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void st_agent(T* p, T v) {
  __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T, typename U>
__device__ inline T g_add(T* p, U v) {
  return __hip_atomic_fetch_add(gp(p), static_cast<T>(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T, typename U>
__device__ inline T g_min(T* p, U v) {
  return __hip_atomic_fetch_min(gp(p), static_cast<T>(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T, typename U>
__device__ inline T g_exch(T* p, U v) {
  return __hip_atomic_exchange(gp(p), static_cast<T>(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// compare-and-swap; returns true when *p held `expected` and now holds `desired`
template <typename T>
__device__ inline bool g_cas(T* p, T expected, T desired) {
  return __hip_atomic_compare_exchange_strong(gp(p), &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
}

// number of set bits of `mask` in lanes below this one
__device__ inline uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ inline uint32_t lane() { return __lane_id(); }

__device__ inline int first_lane(uint64_t mask) { return __ffsll(static_cast<unsigned long long>(mask)) - 1; }

// Append `v` to list[*count] for every lane with `pred`; one atomic per wave.
__device__ inline void push_wave(uint32_t* list, uint32_t* count, bool pred, uint32_t v) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  const int leader = first_lane(mask);
  uint32_t base = 0;
  if (static_cast<int>(lane()) == leader) base = g_add(count, static_cast<uint32_t>(__popcll(mask)));
  base = __shfl(base, leader);
  if (pred) st_agent(&list[base + lanes_below(mask)], v);
}

// Inclusive prefix sum across a wave64.
__device__ inline uint32_t wave_scan(uint32_t x) {
  const uint32_t l = lane();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (l >= static_cast<uint32_t>(d)) x += y;
  }
  return x;
}

// Exclusive prefix sum across a workgroup of WG threads; returns the total in *total.
template <uint32_t WG = kWG>
__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t* total, uint32_t* s_wsum) {
  const uint32_t inc = wave_scan(x);
  const uint32_t w = threadIdx.x >> 6;
  if (lane() == 63) s_wsum[w] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (uint32_t k = 0; k < WG / 64; ++k) {
    const uint32_t s = s_wsum[k];
    before += (k < w) ? s : 0u;
    all += s;
  }
  *total = all;
  __syncthreads();  // s_wsum is reused by the next scan
  return before + inc - x;
}

// ------------------------------------------------------------------ weights

// x (+) w in the weight type, the bucket index floor(x / delta), and the
// weight of the edge record at position pos. T: the distance bits; Wt: the
// weight bits.
struct WeightU32 {
  static constexpr bool kInteger = true;
  static constexpr bool kPacked = true;  // distance words carry the frontier tag (see dist_word)
  using T = uint32_t;
  using Wt = uint32_t;
  static constexpr T kInf = kInfU32;
  __device__ static bool add(T t, Wt w, T* out) {
    const uint64_t s = static_cast<uint64_t>(t) + static_cast<uint64_t>(w);
    *out = static_cast<uint32_t>(s);
    return s <= 0xFFFFFFFEull;  // 2^32-1 is reserved for "unreachable"
  }
  __device__ static uint32_t bucket(T x, const Params& p) { return x / p.delta_u; }
  __device__ static Wt weight(const Params&, uint64_t rec, uint32_t) { return static_cast<Wt>(rec >> 32); }
};

struct WeightF32 {
  static constexpr bool kInteger = false;
  static constexpr bool kPacked = true;
  using T = uint32_t;
  using Wt = uint32_t;
  static constexpr T kInf = kInfF32;
  __device__ static bool add(T t, Wt w, T* out) {
    const float s = __fadd_rn(__uint_as_float(t), __uint_as_float(w));
    *out = __float_as_uint(s);
    return *out < kInfF32;  // non-negative operands: the sum is finite or +inf
  }
  // floor(x / delta) exactly (bucket i holds i*delta <= x < (i+1)*delta): the
  // estimate from one rounded product is off by at most one, and the sign of
  // j*delta - x is exact in a fused multiply-add (one rounding of an exact
  // value, which is zero only when the value is), for every j below 2^32.
  __device__ static uint32_t bucket(T x, const Params& p) {
    const double d = static_cast<double>(__uint_as_float(x));
    double j = floor(d * p.inv_delta_d);
    if (fma(j, p.delta_d, -d) > 0.0) j -= 1.0;
    else if (fma(j + 1.0, p.delta_d, -d) <= 0.0) j += 1.0;
    return static_cast<uint32_t>(j);
  }
  __device__ static Wt weight(const Params&, uint64_t rec, uint32_t) { return static_cast<Wt>(rec >> 32); }
};

struct WeightF64 {
  static constexpr bool kInteger = false;
  static constexpr bool kPacked = false;  // the distance fills the word; the frontier uses qstamp
  using T = uint64_t;
  using Wt = uint64_t;
  static constexpr T kInf = kInfF64;
  __device__ static bool add(T t, Wt w, T* out) {
    const double s = __dadd_rn(__longlong_as_double(static_cast<long long>(t)),
                               __longlong_as_double(static_cast<long long>(w)));
    *out = static_cast<uint64_t>(__double_as_longlong(s));
    return *out < kInfF64;
  }
  // floor(x / delta) exactly, as for fp32 (the sign of the fused j*delta - x
  // is exact: subnormals keep any nonzero difference of doubles nonzero)
  __device__ static uint32_t bucket(T x, const Params& p) {
    const double d = __longlong_as_double(static_cast<long long>(x));
    double j = floor(d * p.inv_delta_d);
    if (fma(j, p.delta_d, -d) > 0.0) j -= 1.0;
    else if (fma(j + 1.0, p.delta_d, -d) <= 0.0) j += 1.0;
    return static_cast<uint32_t>(j);
  }
  __device__ static Wt weight(const Params& p, uint64_t, uint32_t pos) { return ldg(&p.w64[pos]); }
};

// Tentative distances are 64-bit words. For 32-bit distances (u32, fp32 bits)
// the word is (distance << 32) | tag. The tag names the step whose frontier
// last received the vertex in the current bucket: (step << 1) | 1 when queued,
// (step << 1) once the vertex has been expanded at this very distance while
// queued (its queued entry then has nothing new to send), 0 after an update
// that filed it elsewhere. One 64-bit atomic min both decides an update and
// tells whether the vertex is already queued for the next light phase; at an
// equal distance a candidate (queued tag) never replaces a word, since the
// expanded form of the same step sorts below it and earlier steps sort lower
// still. For fp64 the word is the distance alone.
__device__ inline uint32_t queued_tag(uint32_t step) { return (step << 1) | 1u; }
__device__ inline uint32_t tag_step(uint32_t tag) { return tag >> 1; }
__device__ inline bool tag_expanded(uint32_t tag) { return (tag & 1u) == 0u; }
template <class W>
__device__ inline typename W::T word_dist(uint64_t w) {
  if constexpr (W::kPacked) return static_cast<typename W::T>(w >> 32);
  else return w;
}
template <class W>
__device__ inline uint64_t dist_word(typename W::T x, uint32_t tag) {
  if constexpr (W::kPacked) return (static_cast<uint64_t>(x) << 32) | tag;
  else return x;
}
// the distance of v, device-scope
template <class W>
__device__ inline typename W::T tload(const uint64_t* t, uint32_t v) {
  return word_dist<W>(ld_agent(&t[v]));
}
// the distance of v through the caches (possibly stale, never below the current value)
template <class W>
__device__ inline typename W::T tload_cached(const uint64_t* t, uint32_t v) {
  if constexpr (W::kPacked) return ldg(reinterpret_cast<const uint32_t*>(t) + 2 * static_cast<size_t>(v) + 1);
  else return ldg(&t[v]);
}
template <class W>
__device__ inline void tstore(uint64_t* t, uint32_t v, typename W::T x) {
  st_agent(&t[v], dist_word<W>(x, 0u));
}

// ------------------------------------------------------------------ barrier

// Every wave's device-scope stores and atomics complete (are acknowledged by
// the device-coherent level) before its workgroup arrives: s_waitcnt with all
// counters zero.
__device__ inline void drain_stores() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
}

// One record of a traced run (`trace`: the control block's trace buffer, null
// when the run is not traced).
__device__ inline void record_trace(Ctl* c, unsigned long long* trace, uint32_t flags) {
  if (!trace) return;
  const uint32_t idx = g_add(&c->trace_len, 1u);
  if (idx < ldg(&c->trace_cap)) {
    const unsigned long long what = static_cast<unsigned long long>(ld_agent(&c->in_count)) << 32 |
                                    static_cast<unsigned long long>(ld_agent(&c->bucket) & 0xFFFFFFu) << 8 |
                                    (ld_agent(&c->action) | flags);
    st_agent(&trace[4 * idx], static_cast<unsigned long long>(wall_clock64()));
    st_agent(&trace[4 * idx + 1], what);
    st_agent(&trace[4 * idx + 2], g_exch(&c->tr_edges, 0ull));
    st_agent(&trace[4 * idx + 3], g_exch(&c->tr_impr, 0ull));
  }
}

// Barrier over the `size` co-resident workgroups that share the control block
// `c` (this one has index `rank` among them). Arrivals are counted first per
// sub-group (rank % 8), then once per sub-group, which keeps same-address
// atomics short. The last workgroup to arrive runs `leader` (all its threads)
// before releasing the others by advancing the generation word. `b` (LDS) is
// this workgroup's copy of the generation (every workgroup passes every
// barrier, so no load of the word is needed before arriving) and of the trace
// buffer pointer and of the wait limit, loaded by init_barrier at kernel
// start. Returns false when the schedule was aborted: by another workgroup, or
// because a wait saw neither the release nor a new heartbeat of the leader
// (which it bumps at every step it runs alone inside the barrier) for longer
// than the wait limit.
struct BarrierState {
  uint32_t gen;
  unsigned long long* trace;
  unsigned long long wait_ticks;
};

__device__ inline void init_barrier(Ctl* c, BarrierState& b) {
  if (threadIdx.x == 0) {
    b.gen = ld_agent(&c->bar_gen);
    b.trace = ldg(&c->trace);
    b.wait_ticks = ldg(&c->wait_ticks);
  }
  __syncthreads();
}

template <class F>
__device__ bool grid_sync(Ctl* c, uint32_t size, uint32_t rank, BarrierState& b, F&& leader) {
  __shared__ uint32_t s_is_leader;
  __shared__ uint32_t s_ok;
  drain_stores();
  __syncthreads();
  uint32_t gen = 0;
  if (threadIdx.x == 0) {
    const uint32_t groups = size < kBarGroups ? size : kBarGroups;
    const uint32_t g = rank % groups;
    const uint32_t gsize = (size - g + groups - 1) / groups;
    gen = b.gen;
    bool last = false;
    const uint32_t prev = g_add(&c->bar_sub[g][0], 1u);
    if (prev == gsize - 1) {
      st_agent(&c->bar_sub[g][0], 0u);  // the whole group has arrived; nobody re-arrives before the release
      last = g_add(&c->bar_arrive, 1u) == groups - 1;
      if (last) st_agent(&c->bar_arrive, 0u);
    }
    s_is_leader = last ? 1u : 0u;
    uint32_t ok = 1;
    if (!last) {
      // the generation, the abort flag and the heartbeat are loaded together: one round trip per poll
      unsigned long long t0 = wall_clock64();
      uint32_t beat = ld_agent(&c->heartbeat);
      for (;;) {
        const uint32_t g_now = ld_agent(&c->bar_gen);
        const uint32_t abort_now = ld_agent(&c->abort);
        const uint32_t beat_now = ld_agent(&c->heartbeat);
        if (g_now != gen) break;
        if (beat_now != beat) {  // the leader is still making progress
          beat = beat_now;
          t0 = wall_clock64();
        }
        if (abort_now != 0u || wall_clock64() - t0 > b.wait_ticks) {
          st_agent(&c->abort, 1u);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    s_ok = ok;
  }
  __syncthreads();
  if (s_is_leader) {
    if (threadIdx.x == 0) g_add(&c->barriers, 1ull);  // completes with the leader's own stores below
    leader();
    drain_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
      if (b.trace) {
        record_trace(c, b.trace, 0u);
        drain_stores();
      }
      st_agent(&c->bar_gen, gen + 1u);
    }
  }
  const bool ok = s_ok != 0u;
  __syncthreads();
  if (threadIdx.x == 0) b.gen = gen + 1u;
  return ok;
}

}  // namespace
}  // namespace sssp
