// Adjoint of the shortest-path distances with respect to the edge weights:
// for L with dL/dd = grad_dist, dL/dw_e is the sum of grad_dist over the
// subtree hanging below e in each source's shortest-path tree (d(v) is the
// fold of the weights along its tree path). Parents are recomputed from the
// distances (no state is kept from the forward pass):
//   1. every edge out of a reached vertex is checked for feasibility,
//      d(y) <= d(x) (+) w, and d(s) must be +0: with tight parents leading back
//      to s (checked below) this proves that the distances are the shortest
//      ones (Sec. III-C: no relaxation can lower them);
//      the parent of y is its tight in-edge (d(x) (+) w == d(y)) from a
//      strictly closer vertex (d(x) < d(y)) with the smallest caller edge
//      index -- atomicMin over edges. In exact arithmetic every tight edge is
//      of that kind; with rounding, d(x) (+) w can equal d(x) (w absorbed), so
//      a vertex may be tight only through in-edges from vertices at its own
//      distance, which can form cycles. Those vertices are resolved in rounds:
//      round 0 holds s and the vertices with a strictly closer parent; round k
//      gives each unresolved vertex the smallest-index tight in-edge from a
//      vertex resolved in round k - 1;
//   2. children are counted; vertices without children form the first level;
//   3. level by level, each vertex adds its accumulated value g(v) to its
//      parent edge and to g(parent) (fp64 atomics); a parent whose last child
//      has reported joins the next level.
// One cooperative launch handles all sources; dL/dw is accumulated in fp64
// over the sources and written as fp32 in the caller's edge order.
#include "sssp_device.h"

namespace sssp {
namespace {

constexpr unsigned long long kNoParent = ~0ull;

template <class W>
__device__ void adjoint_leader_level(Ctl* c, uint32_t cur) {
  if (threadIdx.x == 0) {
    const uint32_t nxt = 1u - cur;
    st_agent(&c->in_count, ld_agent(&c->fcount[nxt]));
    st_agent(&c->fcount[cur], 0u);
    st_agent(&c->out_buf, nxt);
  }
}

// The count gathered in scount by the step that just ended becomes in_count
// (read by every workgroup after the barrier); scount restarts at zero.
__device__ inline void adjoint_leader_count(Ctl* c) {
  if (threadIdx.x == 0) {
    st_agent(&c->in_count, ld_agent(&c->scount));
    st_agent(&c->scount, 0u);
  }
}

template <class W>
__global__ __launch_bounds__(kWG) void adjoint_kernel(const AdjParams* __restrict__ params, uint32_t groups,
                                                      const int32_t* sources, int k, const uint32_t* dist,
                                                      const float* grad_dist) {
  // workgroup b belongs to group b % groups; each group handles one source at a time
  const AdjParams& a = params[blockIdx.x % groups];
  const uint32_t rank = blockIdx.x / groups, size = gridDim.x / groups;
  Ctl* c = a.ctl;
  const uint32_t n = a.n;
  const uint32_t tid = rank * kWG + threadIdx.x;
  const uint32_t nthreads = size * kWG;
  __shared__ uint32_t s_count, s_cur, s_row;
  __shared__ BarrierState s_bar;
  init_barrier(c, s_bar);
  bool alive = true;
  while (alive) {
    // claim the next source row for this group
    alive = grid_sync(c, size, rank, s_bar, [&] {
      if (threadIdx.x == 0) {
        const uint32_t r = g_add(a.next_source, 1u);
        st_agent(&c->source_index, r < static_cast<uint32_t>(k) ? r : kNone);
        st_agent(&c->fcount[0], 0u);
        st_agent(&c->fcount[1], 0u);
        st_agent(&c->scount, 0u);
      }
    });
    if (threadIdx.x == 0) s_row = ld_agent(&c->source_index);
    __syncthreads();
    const uint32_t r = s_row;
    if (!alive || r == kNone) break;
    const int32_t src = ldg(&sources[r]);
    if (src < 0 || static_cast<uint32_t>(src) >= n) {  // every workgroup of the group skips the row
      if (rank == 0 && threadIdx.x == 0) st_agent(&c->bad_source, 1u);
      continue;
    }
    const uint32_t* drow = dist + static_cast<size_t>(r) * n;
    const float* grow = grad_dist + static_cast<size_t>(r) * n;
    const uint32_t s = ldg(&a.vid[src]);
    // distances and coefficients in solver ids
    for (uint32_t x = tid; x < n; x += nthreads) {
      const uint32_t v = ldg(&a.inv[x]);
      const uint32_t dx = ldg(&drow[v]);
      st_agent(&a.d[x], dx);
      st_agent(&a.parent[x], kNoParent);
      st_agent(&a.cnt[x], 0u);
      st_agent(&a.g[x], (dx < W::kInf && x != s) ? static_cast<double>(ldg(&grow[v])) : 0.0);
      if (x == s && dx != 0u) st_agent(&c->ovf_real, 1u);  // d(s) must be +0
    }
    alive = grid_sync(c, size, rank, s_bar, [] {});
    if (!alive) break;
    // 1. feasibility, and parents from strictly closer vertices: one wave per row, lanes over its edges
    {
      const uint32_t wave = tid >> 6, nwaves = nthreads >> 6, l = lane();
      for (uint32_t x = wave; x < n; x += nwaves) {
        const uint32_t dx = ld_agent(&a.d[x]);
        if (dx >= W::kInf) continue;
        const uint4 row = ldg(&a.rows[x]);
        bool infeasible = false;
        for (uint32_t p = row.x + l; p < row.z; p += 64) {
          const uint64_t ed = ldg(&a.edges[p]);
          const uint32_t y = static_cast<uint32_t>(ed);
          uint32_t cand;
          if (!W::add(dx, static_cast<uint32_t>(ed >> 32), &cand)) continue;  // the request does not fit: no bound
          const uint32_t dy = ld_agent(&a.d[y]);
          if (dy > cand) infeasible = true;  // an edge could still lower d(y)
          else if (cand == dy && dx < dy && y != s)
            g_min(&a.parent[y], static_cast<unsigned long long>(ldg(&a.perm[p])) << 32 | x);
        }
        if (__ballot(infeasible) && l == 0) st_agent(&c->ovf_real, 1u);
      }
    }
    alive = grid_sync(c, size, rank, s_bar, [] {});
    if (!alive) break;
    // 1b. round 0: s and the vertices with a strictly closer parent; the other reached vertices are unresolved
    for (uint32_t it = 0, iters = (n + nthreads - 1) / nthreads; it < iters; ++it) {
      const uint32_t y = it * nthreads + tid;
      bool open = false;
      if (y < n) {
        open = y != s && ld_agent(&a.d[y]) < W::kInf && ld_agent(&a.parent[y]) == kNoParent;
        st_agent(&a.lvl[y], open ? kNone : 0u);
      }
      const uint32_t cnt = static_cast<uint32_t>(__popcll(__ballot(open)));
      if (cnt && lane() == 0) g_add(&c->scount, cnt);
    }
    alive = grid_sync(c, size, rank, s_bar, [&] { adjoint_leader_count(c); });
    // 1c. rounds k = 1, 2, ... while unresolved vertices gain a parent
    for (uint32_t rnd = 1; alive; ++rnd) {
      if (threadIdx.x == 0) s_count = ld_agent(&c->in_count);
      __syncthreads();
      if (s_count == 0) break;
      {
        const uint32_t wave = tid >> 6, nwaves = nthreads >> 6, l = lane();
        for (uint32_t x = wave; x < n; x += nwaves) {
          if (ld_agent(&a.lvl[x]) != rnd - 1) continue;
          const uint32_t dx = ld_agent(&a.d[x]);
          if (dx >= W::kInf) continue;
          const uint4 row = ldg(&a.rows[x]);
          for (uint32_t p = row.x + l; p < row.z; p += 64) {
            const uint64_t ed = ldg(&a.edges[p]);
            const uint32_t y = static_cast<uint32_t>(ed);
            uint32_t cand;
            if (ld_agent(&a.lvl[y]) == kNone && W::add(dx, static_cast<uint32_t>(ed >> 32), &cand) &&
                cand == ld_agent(&a.d[y]))
              g_min(&a.parent[y], static_cast<unsigned long long>(ldg(&a.perm[p])) << 32 | x);
          }
        }
      }
      alive = grid_sync(c, size, rank, s_bar, [] {});
      if (!alive) break;
      for (uint32_t it = 0, iters = (n + nthreads - 1) / nthreads; it < iters; ++it) {
        const uint32_t y = it * nthreads + tid;
        bool grew = false;
        if (y < n && ld_agent(&a.lvl[y]) == kNone && ld_agent(&a.parent[y]) != kNoParent) {
          st_agent(&a.lvl[y], rnd);
          grew = true;
        }
        const uint32_t cnt = static_cast<uint32_t>(__popcll(__ballot(grew)));
        if (cnt && lane() == 0) g_add(&c->scount, cnt);
      }
      alive = grid_sync(c, size, rank, s_bar, [&] { adjoint_leader_count(c); });
    }
    if (!alive) break;
    // 2. children per vertex; a reached vertex other than s must have a parent
    for (uint32_t y = tid; y < n; y += nthreads) {
      if (y == s || ld_agent(&a.d[y]) >= W::kInf) continue;
      const unsigned long long pe = ld_agent(&a.parent[y]);
      if (pe == kNoParent) st_agent(&c->ovf_real, 1u);  // not a shortest-path vector
      else g_add(&a.cnt[static_cast<uint32_t>(pe)], 1u);
    }
    alive = grid_sync(c, size, rank, s_bar, [] {});
    if (!alive) break;
    // 3. first level: reached vertices without children
    {
      const uint32_t iters = (n + nthreads - 1) / nthreads;
      for (uint32_t it = 0; it < iters; ++it) {
        const uint32_t y = it * nthreads + tid;
        const bool leaf = y < n && ld_agent(&a.d[y]) < W::kInf && ld_agent(&a.cnt[y]) == 0u;
        push_wave(a.front[0], &c->fcount[0], leaf, y);
      }
    }
    alive = grid_sync(c, size, rank, s_bar, [&] { adjoint_leader_level<W>(c, 1u); });  // in_count = fcount[0], out = 0
    // 4. levels, leaves towards the source
    while (alive) {
      if (threadIdx.x == 0) {
        s_count = ld_agent(&c->in_count);
        s_cur = ld_agent(&c->out_buf);
      }
      __syncthreads();
      const uint32_t count = s_count, cur = s_cur, nxt = 1u - cur;
      if (count == 0) break;
      const uint32_t iters = (count + nthreads - 1) / nthreads;
      uint32_t released = 0;
      for (uint32_t it = 0; it < iters; ++it) {
        const uint32_t i = it * nthreads + tid;
        bool up = false;
        uint32_t x = 0;
        if (i < count) {
          const uint32_t y = ld_agent(&a.front[cur][i]);
          ++released;
          const unsigned long long pe = y != s ? ld_agent(&a.parent[y]) : kNoParent;
          if (pe != kNoParent) {  // (a reached vertex without a parent was reported above)
            x = static_cast<uint32_t>(pe);
            const double gy = ld_agent(&a.g[y]);
            g_add(&a.grad64[pe >> 32], gy);
            g_add(&a.g[x], gy);  // read by x's own level, after the next barrier
            up = g_add(&a.cnt[x], 0xFFFFFFFFu) == 1u;  // the last child to report releases the parent
          }
        }
        push_wave(a.front[nxt], &c->fcount[nxt], up, x);
      }
      // every reached vertex is released exactly once unless the parents form a cycle
      if (released) g_add(&c->adj_released, static_cast<unsigned long long>(released));
      alive = grid_sync(c, size, rank, s_bar, [&] { adjoint_leader_level<W>(c, cur); });
    }
  }
}

// dL/dw in the caller's edge order, from the fp64 accumulator
__global__ __launch_bounds__(kAuxWG) void grad_to_f32_kernel(const double* g64, uint64_t m, float* out) {
  for (uint64_t e = static_cast<uint64_t>(blockIdx.x) * kAuxWG + threadIdx.x; e < m;
       e += static_cast<uint64_t>(gridDim.x) * kAuxWG)
    out[e] = static_cast<float>(g64[e]);
}

// Number of reached vertices of a distance row (for the release-count check).
template <class W>
__global__ __launch_bounds__(kAuxWG) void count_reached_kernel(const uint32_t* dist, uint32_t n, int k,
                                                               unsigned long long* out) {
  unsigned long long cnt = 0;
  const size_t total = static_cast<size_t>(n) * k;
  for (size_t i = static_cast<size_t>(blockIdx.x) * kAuxWG + threadIdx.x; i < total;
       i += static_cast<size_t>(gridDim.x) * kAuxWG)
    cnt += dist[i] < W::kInf ? 1u : 0u;
  for (int d = 32; d > 0; d >>= 1) cnt += __shfl_down(cnt, d);
  if (lane() == 0 && cnt) atomicAdd(out, cnt);
}

// Re-split with new weights: one wave per solver row re-partitions the row's
// records (light first, then heavy; each group keeps the records' current
// order) with the new weight of each record's caller edge.
__global__ __launch_bounds__(kAuxWG) void resplit_kernel(uint32_t n, const uint4* rows_in, const uint64_t* edges_in,
                                                         const uint32_t* perm_in, const void* w, Threshold th,
                                                         uint4* rows_out, uint64_t* w64_out, uint64_t* edges_out,
                                                         uint32_t* perm_out) {
  const uint32_t wave = (blockIdx.x * kAuxWG + threadIdx.x) >> 6;
  const uint32_t nwaves = (gridDim.x * kAuxWG) >> 6;
  const uint32_t l = lane();
  for (uint32_t x = wave; x < n; x += nwaves) {
    const uint4 row = rows_in[x];
    uint32_t nlight = 0;
    for (uint32_t p = row.x; p < row.z; p += 64) {
      bool light = false;
      if (p + l < row.z) light = is_light(weight_bits(w, th.wtype, perm_in[p + l]), th);
      nlight += static_cast<uint32_t>(__popcll(__ballot(light)));
    }
    if (l == 0) rows_out[x] = make_uint4(row.x, row.x + nlight, row.z, 0u);
    uint32_t lpos = row.x, hpos = row.x + nlight;
    for (uint32_t p = row.x; p < row.z; p += 64) {
      const bool in = p + l < row.z;
      bool light = false;
      uint64_t wb = 0;
      uint32_t y = 0, ce = 0;
      if (in) {
        ce = perm_in[p + l];
        y = static_cast<uint32_t>(edges_in[p + l]);
        wb = weight_bits(w, th.wtype, ce);
        light = is_light(wb, th);
      }
      const uint64_t ml = __ballot(in && light);
      const uint64_t mh = __ballot(in && !light);
      if (in) {
        const uint32_t pos = light ? lpos + lanes_below(ml) : hpos + lanes_below(mh);
        if (th.wtype == kWF64) {
          edges_out[pos] = static_cast<uint64_t>(y);
          w64_out[pos] = wb;
        } else {
          edges_out[pos] = static_cast<uint64_t>(y) | (wb << 32);
        }
        perm_out[pos] = ce;
      }
      lpos += static_cast<uint32_t>(__popcll(ml));
      hpos += static_cast<uint32_t>(__popcll(mh));
    }
  }
}

}  // namespace

hipError_t adjoint_occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, adjoint_kernel<WeightF32>, kWG, 0);
}

hipError_t launch_adjoint(const AdjParams* params, uint32_t groups, const int32_t* sources, int k, const uint32_t* dist,
                          const float* grad_dist, float* grad_w, uint64_t m, double* grad64, int grid, hipStream_t s) {
  if (groups < 1 || groups > kMaxGroups || grid < 1 || grid % static_cast<int>(groups) != 0) return hipErrorInvalidValue;
  hipError_t e = launch_fill(reinterpret_cast<uint32_t*>(grad64), 2 * static_cast<size_t>(m), 0u, s);
  if (e != hipSuccess) return e;
  const AdjParams* pp = params;
  uint32_t gg = groups;
  const int32_t* src = sources;
  int kk = k;
  const uint32_t* d = dist;
  const float* gd = grad_dist;
  void* args[] = {&pp, &gg, &src, &kk, &d, &gd};
  e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(adjoint_kernel<WeightF32>), dim3(grid), dim3(kWG), args,
                                 0, s);
  if (e != hipSuccess) return e;
  size_t blocks = (static_cast<size_t>(m) + kAuxWG - 1) / kAuxWG;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(grad_to_f32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kAuxWG), 0, s, grad64, m, grad_w);
  return hipGetLastError();
}

hipError_t launch_count_reached(const uint32_t* dist, uint32_t n, int k, int wtype, unsigned long long* out,
                                hipStream_t s) {
  const size_t total = static_cast<size_t>(n) * k;
  size_t blocks = (total + kAuxWG - 1) / kAuxWG;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  if (wtype == 0)
    hipLaunchKernelGGL(count_reached_kernel<WeightU32>, dim3(static_cast<unsigned>(blocks)), dim3(kAuxWG), 0, s, dist,
                       n, k, out);
  else
    hipLaunchKernelGGL(count_reached_kernel<WeightF32>, dim3(static_cast<unsigned>(blocks)), dim3(kAuxWG), 0, s, dist,
                       n, k, out);
  return hipGetLastError();
}

hipError_t launch_resplit(uint32_t n, const uint4* rows_in, const uint64_t* edges_in, const uint32_t* perm_in,
                          const void* w, const Threshold& th, uint4* rows_out, uint64_t* w64_out,
                          uint64_t* edges_out, uint32_t* perm_out, hipStream_t s) {
  size_t blocks = (static_cast<size_t>(n) * 64 + kAuxWG - 1) / kAuxWG;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(resplit_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kAuxWG), 0, s, n, rows_in, edges_in,
                     perm_in, w, th, rows_out, w64_out, edges_out, perm_out);
  return hipGetLastError();
}

}  // namespace sssp
