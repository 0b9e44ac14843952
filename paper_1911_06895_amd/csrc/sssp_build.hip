// Create-time kernels: validation of the caller's CSR, the vertex relabelling
// that lays distances out for the L2 caches, and the light/heavy split of the
// adjacency matrix (Sec. IV-A) into the solver's packed edge records.
//
// Relabelling: the solver gathers t(v) once per edge into v, so the hot part of
// t is the set of vertices with many in-edges. Vertices are renumbered by
// decreasing in-degree; on power-law graphs the distances that absorb most
// relaxations then share a few megabytes that each XCD's L2 keeps resident.
// Distances are translated back to the caller's numbering when a solve ends.
#include "sssp_internal.h"

namespace sssp {
namespace {

constexpr int kB = kAuxWG;
constexpr uint32_t kScanItems = 4;                    // entries per thread in the scan kernels
constexpr uint32_t kScanTile = kB * kScanItems;       // entries per scan block

__device__ inline uint32_t lane_id() { return __lane_id(); }

__device__ inline uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ inline uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (l >= static_cast<uint32_t>(d)) x += y;
  }
  return x;
}

// exclusive scan across a kB-thread block; *total receives the block sum
__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t* total) {
  __shared__ uint32_t s_w[kB / 64];
  const uint32_t inc = wave_incl_scan(x);
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 63) s_w[w] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (uint32_t k = 0; k < kB / 64; ++k) {
    before += k < w ? s_w[k] : 0u;
    all += s_w[k];
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

// Per-wave fold of the weight checks into the outputs.
__device__ inline void fold_weights(uint32_t bad, unsigned long long wmax, double sum, uint32_t* status,
                                    unsigned long long* wmax_bits, double* wsum) {
  for (int d = 32; d > 0; d >>= 1) {
    bad |= __shfl_down(bad, d);
    wmax = max(wmax, __shfl_down(wmax, d));
    sum += __shfl_down(sum, d);
  }
  if (lane_id() == 0) {
    if (bad) atomicOr(status, bad);
    if (wmax) atomicMax(wmax_bits, wmax);
    if (sum != 0.0) atomicAdd(wsum, sum);
  }
}

// CSR and weight validation; the largest weight (as bits: positive floats
// order like their bit patterns) and the weight total, for the bucket-range check.
__global__ __launch_bounds__(kB) void validate_kernel(const int64_t* rp, const int32_t* col, const void* w,
                                                      int wtype, int64_t n, int64_t m, uint32_t* status,
                                                      unsigned long long* wmax_bits, double* wsum) {
  uint32_t bad = 0;
  unsigned long long wmax = 0;
  double sum = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kB;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  for (int64_t u = i0; u <= n; u += stride) {
    const int64_t a = rp[u];
    if (u == 0 && a != 0) bad |= kBadRowPtr;
    if (u == n && a != m) bad |= kBadRowPtr;
    if (u < n && rp[u + 1] < a) bad |= kBadRowPtr;
  }
  for (int64_t e = i0; e < m; e += stride) {
    const int32_t c = col[e];
    if (c < 0 || c >= n) bad |= kBadCol;
    const uint64_t wb = weight_bits(w, wtype, e);
    if (!weight_ok(wb, wtype)) bad |= kBadWeight;
    else sum += weight_value(wb, wtype);
    wmax = max(wmax, static_cast<unsigned long long>(wb));
  }
  fold_weights(bad, wmax, sum, status, wmax_bits, wsum);
}

// weights only (used when a handle's weights are replaced)
__global__ __launch_bounds__(kB) void validate_weights_kernel(const void* w, int wtype, int64_t m, uint32_t* status,
                                                              unsigned long long* wmax_bits, double* wsum) {
  uint32_t bad = 0;
  unsigned long long wmax = 0;
  double sum = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kB;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x; e < m; e += stride) {
    const uint64_t wb = weight_bits(w, wtype, e);
    if (!weight_ok(wb, wtype)) bad |= kBadWeight;
    else sum += weight_value(wb, wtype);
    wmax = max(wmax, static_cast<unsigned long long>(wb));
  }
  fold_weights(bad, wmax, sum, status, wmax_bits, wsum);
}

__global__ __launch_bounds__(kB) void inverse_kernel(const uint32_t* vid, int64_t n, uint32_t* inv) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kB;
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x; v < n; v += stride)
    inv[vid[v]] = static_cast<uint32_t>(v);
}

// in-degree of every vertex (col is validated)
__global__ __launch_bounds__(kB) void indegree_kernel(const int32_t* col, int64_t m, uint32_t* indeg) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kB;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x; e < m; e += stride)
    atomicAdd(&indeg[col[e]], 1u);
}

__device__ inline uint32_t degree_class(uint32_t d) { return d < kDegClasses - 1 ? d : kDegClasses - 1; }

// Lanes of a wave holding the same key form a group; returns this lane's group
// (as a lane mask) and its leader, with ballots only. Degree classes are very
// unequal in size, so one atomic per group instead of per lane avoids long
// same-address queues.
__device__ inline uint64_t group_by_key(bool active, uint32_t key, int* leader) {
  uint64_t rest = __ballot(active), mine = 0;
  *leader = 0;
  while (rest) {
    const int l = __ffsll(static_cast<unsigned long long>(rest)) - 1;
    const uint32_t kl = __builtin_amdgcn_readlane(key, l);
    const bool same = active && key == kl;
    const uint64_t grp = __ballot(same);
    if (same) {
      mine = grp;
      *leader = l;
    }
    rest &= ~grp;
  }
  return mine;
}

__global__ __launch_bounds__(kB) void degree_histogram_kernel(const uint32_t* indeg, int64_t n, uint32_t* hist) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kB;
  const int64_t iters = (n + stride - 1) / stride;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t v = it * stride + static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
    const bool active = v < n;
    const uint32_t c = active ? degree_class(indeg[v]) : 0u;
    int leader;
    const uint64_t grp = group_by_key(active, c, &leader);
    if (active && static_cast<int>(lane_id()) == leader) atomicAdd(&hist[c], static_cast<uint32_t>(__popcll(grp)));
  }
}

// cursor[d] = number of vertices in higher degree classes (one block)
__global__ __launch_bounds__(kB) void class_start_kernel(const uint32_t* hist, uint32_t* cursor) {
  constexpr uint32_t per = kDegClasses / kB;
  // thread k owns classes (in decreasing order) k*per .. k*per+per-1 counted from the top
  uint32_t local = 0;
  for (uint32_t i = 0; i < per; ++i) local += hist[kDegClasses - 1 - (threadIdx.x * per + i)];
  uint32_t total;
  uint32_t run = block_excl_scan(local, &total);
  for (uint32_t i = 0; i < per; ++i) {
    const uint32_t d = kDegClasses - 1 - (threadIdx.x * per + i);
    cursor[d] = run;
    run += hist[d];
  }
}

// new id of every vertex: position in decreasing degree class order
__global__ __launch_bounds__(kB) void assign_ids_kernel(const uint32_t* indeg, int64_t n, uint32_t* cursor,
                                                        uint32_t* new_id) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kB;
  const int64_t iters = (n + stride - 1) / stride;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t v = it * stride + static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
    const bool active = v < n;
    const uint32_t c = active ? degree_class(indeg[v]) : 0u;
    int leader;
    const uint64_t grp = group_by_key(active, c, &leader);
    uint32_t base = 0;
    if (active && static_cast<int>(lane_id()) == leader) base = atomicAdd(&cursor[c], static_cast<uint32_t>(__popcll(grp)));
    base = __shfl(base, leader);
    if (active) new_id[v] = base + lanes_below(grp);
  }
}

// out-degree of each vertex, stored at its new id
__global__ __launch_bounds__(kB) void renumbered_outdeg_kernel(const int64_t* rp, const uint32_t* new_id, int64_t n,
                                                               uint32_t* deg) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kB;
  for (int64_t u = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x; u < n; u += stride)
    deg[new_id[u]] = static_cast<uint32_t>(rp[u + 1] - rp[u]);
}

// three-pass exclusive scan of n entries: tile sums, scan of the tile sums, tiles
__global__ __launch_bounds__(kB) void scan_tiles_kernel(const uint32_t* in, int64_t n, uint32_t* tile_sum) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
  uint32_t s = 0;
  for (uint32_t i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  uint32_t total;
  (void)block_excl_scan(s, &total);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kB) void scan_tile_sums_kernel(uint32_t* tile_sum, uint32_t ntiles) {
  __shared__ uint32_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (uint32_t b = 0; b < ntiles; b += kB) {
    const uint32_t i = b + threadIdx.x;
    const uint32_t x = i < ntiles ? tile_sum[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan(x, &total);
    if (i < ntiles) tile_sum[i] = s_carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) s_carry += total;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kB) void scan_apply_kernel(const uint32_t* in, int64_t n, const uint32_t* tile_off,
                                                        uint32_t* out) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems], s = 0;
  for (uint32_t i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t total;
  uint32_t run = tile_off[blockIdx.x] + block_excl_scan(s, &total);
  for (uint32_t i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kB - 1) out[n] = run;  // the grand total
}

// Light/heavy split (Sec. IV-A) with relabelling: one wave per original row u
// writes row new_id[u] of the solver's CSR -- light edges (w <= delta) first,
// heavy edges (w > delta) after, each group in the caller's order -- as packed
// (new destination id | weight bits << 32) records (fp64: the destination,
// and the weight at the same position of w64); perm maps a position back to
// the caller's edge index.
__global__ __launch_bounds__(kB) void split_kernel(const int64_t* rp, const int32_t* col, const void* w, Threshold th,
                                                   int64_t n, const uint32_t* new_id, const uint32_t* off,
                                                   uint32_t* split, uint64_t* edges, uint64_t* w64, uint32_t* perm) {
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * kB) >> 6;
  const uint32_t l = lane_id();
  for (int64_t u = wave; u < n; u += nwaves) {
    const int64_t b = rp[u], e = rp[u + 1];
    const uint32_t nu = new_id[u];
    const uint32_t base = off[nu];
    uint32_t nlight = 0;
    for (int64_t x = b; x < e; x += 64) {
      bool light = false;
      if (x + l < e) light = is_light(weight_bits(w, th.wtype, x + l), th);
      nlight += static_cast<uint32_t>(__popcll(__ballot(light)));
    }
    if (l == 0) split[nu] = base + nlight;
    uint32_t lpos = base, hpos = base + nlight;
    for (int64_t x = b; x < e; x += 64) {
      const bool in = x + l < e;
      bool light = false;
      uint64_t wb = 0;
      uint32_t c = 0;
      if (in) {
        wb = weight_bits(w, th.wtype, x + l);
        c = new_id[col[x + l]];
        light = is_light(wb, th);
      }
      const uint64_t ml = __ballot(in && light);
      const uint64_t mh = __ballot(in && !light);
      if (in) {
        const uint32_t pos = light ? lpos + lanes_below(ml) : hpos + lanes_below(mh);
        if (th.wtype == kWF64) {
          edges[pos] = static_cast<uint64_t>(c);
          w64[pos] = wb;
        } else {
          edges[pos] = static_cast<uint64_t>(c) | (wb << 32);
        }
        perm[pos] = static_cast<uint32_t>(x + l);
      }
      lpos += static_cast<uint32_t>(__popcll(ml));
      hpos += static_cast<uint32_t>(__popcll(mh));
    }
  }
}

// one 16-byte record per row for the solver: a single load gives both ranges
__global__ __launch_bounds__(kB) void pack_rows_kernel(const uint32_t* off, const uint32_t* split, int64_t n,
                                                       uint4* rows) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kB;
  for (int64_t u = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x; u < n; u += stride)
    rows[u] = make_uint4(off[u], split[u], off[u + 1], 0u);
}

unsigned grid_for(int64_t work, int64_t cap) {
  int64_t b = (work + kB - 1) / kB;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

}  // namespace

hipError_t launch_validate(const int64_t* row_ptr, const int32_t* col, const void* w, int wtype, int64_t n,
                           int64_t m, uint32_t* status, unsigned long long* wmax_bits, double* wsum, hipStream_t s) {
  hipLaunchKernelGGL(validate_kernel, dim3(grid_for(m > n + 1 ? m : n + 1, 8192)), dim3(kB), 0, s, row_ptr, col, w,
                     wtype, n, m, status, wmax_bits, wsum);
  return hipGetLastError();
}

hipError_t launch_pack_rows(const uint32_t* off, const uint32_t* split, int64_t n, uint4* rows, hipStream_t s) {
  hipLaunchKernelGGL(pack_rows_kernel, dim3(grid_for(n, 8192)), dim3(kB), 0, s, off, split, n, rows);
  return hipGetLastError();
}

hipError_t launch_validate_weights(const void* w, int wtype, int64_t m, uint32_t* status,
                                   unsigned long long* wmax_bits, double* wsum, hipStream_t s) {
  hipLaunchKernelGGL(validate_weights_kernel, dim3(grid_for(m, 8192)), dim3(kB), 0, s, w, wtype, m, status, wmax_bits,
                     wsum);
  return hipGetLastError();
}

hipError_t launch_inverse(const uint32_t* vid, int64_t n, uint32_t* inv, hipStream_t s) {
  hipLaunchKernelGGL(inverse_kernel, dim3(grid_for(n, 8192)), dim3(kB), 0, s, vid, n, inv);
  return hipGetLastError();
}

size_t build_scratch_words(int64_t n) {
  const size_t tiles = static_cast<size_t>((n + kScanTile - 1) / kScanTile) + 1;
  return static_cast<size_t>(n) /* indeg, then renumbered out-degree */ + kDegClasses * 2 + tiles;
}

hipError_t launch_relabel_and_split(const int64_t* row_ptr, const int32_t* col, const void* w, const Threshold& th,
                                    int64_t n, int64_t m, uint32_t* scratch, uint32_t* new_id, uint32_t* off,
                                    uint32_t* split, uint64_t* edges, uint64_t* w64, uint32_t* perm, hipStream_t s) {
  uint32_t* indeg = scratch;               // [n]
  uint32_t* hist = scratch + n;            // [kDegClasses]
  uint32_t* cursor = hist + kDegClasses;   // [kDegClasses]
  uint32_t* tiles = cursor + kDegClasses;  // [ntiles]
  const uint32_t ntiles = static_cast<uint32_t>((n + kScanTile - 1) / kScanTile);
  hipError_t e = hipMemsetAsync(scratch, 0, (static_cast<size_t>(n) + 2 * kDegClasses) * sizeof(uint32_t), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(indegree_kernel, dim3(grid_for(m, 16384)), dim3(kB), 0, s, col, m, indeg);
  hipLaunchKernelGGL(degree_histogram_kernel, dim3(grid_for(n, 8192)), dim3(kB), 0, s, indeg, n, hist);
  hipLaunchKernelGGL(class_start_kernel, dim3(1), dim3(kB), 0, s, hist, cursor);
  hipLaunchKernelGGL(assign_ids_kernel, dim3(grid_for(n, 8192)), dim3(kB), 0, s, indeg, n, cursor, new_id);
  // the in-degrees are no longer needed: reuse them for the renumbered out-degrees
  hipLaunchKernelGGL(renumbered_outdeg_kernel, dim3(grid_for(n, 8192)), dim3(kB), 0, s, row_ptr, new_id, n, indeg);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3(ntiles), dim3(kB), 0, s, indeg, n, tiles);
  hipLaunchKernelGGL(scan_tile_sums_kernel, dim3(1), dim3(kB), 0, s, tiles, ntiles);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(ntiles), dim3(kB), 0, s, indeg, n, tiles, off);
  const int64_t waves_blocks = (n * 64 + kB - 1) / kB;
  hipLaunchKernelGGL(split_kernel, dim3(static_cast<unsigned>(waves_blocks > 16384 ? 16384 : waves_blocks)),
                     dim3(kB), 0, s, row_ptr, col, w, th, n, new_id, off, split, edges, w64, perm);
  (void)m;
  return hipGetLastError();
}

}  // namespace sssp
