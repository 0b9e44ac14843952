// Host side of the C ABI declared in include/sssp.h: argument checks, device
// memory of a handle, the create-time validation and split, and the solve
// launch with its status read-back.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include <mutex>

#include "sssp.h"
#include "sssp_internal.h"

namespace {
// Fixed working memory of sssp_backward_noalloc: 64 MiB per GPU, held by every
// device the library runs on until the process ends. Every call on one GPU
// shares it (calls that overlap on one GPU race).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the scratch array on `device`, which must be current: each
// GPU holds its own copy at its own address. In host code the array's name is
// only a stand-in, so kernels receive this address, never the name.
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}

size_t align256(size_t bytes) { return (bytes + 255) & ~static_cast<size_t>(255); }
}  // namespace

// Working set of one extra concurrent group (the first group's lives in Params).
struct GroupMem {
  void* tbuf[2] = {nullptr, nullptr};
  void* texp = nullptr;
  uint32_t *qstamp = nullptr, *sstamp = nullptr, *bstamp = nullptr, *fstamp = nullptr, *ovf_at = nullptr;
  uint32_t* front[2] = {nullptr, nullptr};
  uint32_t* slist = nullptr;
  uint32_t* bins = nullptr;
  uint32_t* far[2] = {nullptr, nullptr};
  uint64_t* hub = nullptr;
};

struct sssp_handle {
  int device = 0;
  int64_t n = 0, m = 0;
  int32_t wtype = 0;
  double delta = 0;
  uint32_t delta_u = 0;
  float delta_f = 0;
  double delta_d = 0;
  uint64_t wmax_bits = 0;
  uint64_t* w64 = nullptr;  // [m] fp64 weights at the split positions (fp64 handles)
  int grid = 0;         // workgroups of a launch of one source at a time (kWG threads each)
  int grid_groups = 0;  // workgroups of a launch of concurrent sources (kWGGroups threads, two per CU; 0: none)
  int cus = 0;
  int wallclock_khz = 100000;  // device wall-clock rate (wall_clock64 ticks per millisecond)
  int occupancy = 0;         // co-resident solver workgroups per CU (kWG; the lower of the two kernels)
  int occupancy_groups = 0;  // the same for kWGGroups
  bool chain = false;        // launch the solver whose leader chains its light steps
  sssp_tuning tuning{};
  sssp::Params p{};
  uint32_t* perm = nullptr;
  uint32_t* off = nullptr;    // [n+1] row starts of the split copy (solver ids)
  uint32_t* split = nullptr;  // [n] end of each row's light edges
  int32_t* src_dev = nullptr;
  int32_t src_cap = 0;
  int32_t* src_host = nullptr;   // pinned staging for sources
  sssp::Ctl* ctl_host = nullptr;  // pinned copy of the control blocks [kMaxGroups]
  sssp::Ctl* ctls = nullptr;      // [kMaxGroups] control blocks; group g uses ctls[g]
  sssp::Params* params_dev = nullptr;  // [kMaxGroups + 1] per-group launch parameters; the last: one group alone
  uint32_t groups = 1;            // concurrent groups of the next launch
  uint32_t enq_groups = 0;        // groups of the last enqueued launch (0: none)
  std::vector<GroupMem> extra;    // working sets of groups 1, 2, ...
  sssp_stats last{};
  bool solved = false;
  bool stamps_dirty = false;
  unsigned long long* trace = nullptr;  // caller-owned device buffer (optional)
  uint32_t trace_cap = 0;
  uint32_t* inv = nullptr;  // [n] solver id -> caller id
  // adjoint working set, allocated on first use
  uint32_t* adj_d = nullptr;
  unsigned long long* adj_parent = nullptr;
  uint32_t* adj_cnt = nullptr;
  uint32_t* adj_lvl = nullptr;
  double* adj_g = nullptr;
  double* adj_grad64 = nullptr;
  struct AdjMem {  // adjoint working set of an extra concurrent group
    uint32_t* d = nullptr;
    unsigned long long* parent = nullptr;
    uint32_t* cnt = nullptr;
    uint32_t* lvl = nullptr;
    double* g = nullptr;
  };
  std::vector<AdjMem> adj_extra;
  sssp::AdjParams* adj_params_dev = nullptr;  // [kMaxGroups]
  sssp::AdjParams adj_host[sssp::kMaxGroups];  // host copy of the groups' adjoint launch parameters
  unsigned long long* aux = nullptr;       // [2] small device scratch for status reads
  unsigned long long* aux_host = nullptr;  // [2] pinned host copy of aux
  int adj_grid = 0;
  void* scratch = nullptr;  // this device's copy of the library's static scratch array (sssp_backward_noalloc)
};

namespace {

constexpr uint32_t kDefaultInlineEdges = 4096;
// By default the leader chains its light steps on graphs of low mean out-degree
// (meshes, road-like graphs: long runs of small light phases); on denser graphs
// the chains are short and the plain kernel is as fast.
constexpr int64_t kChainMaxMeanDegree = 6;
constexpr int32_t kDefaultWaitLimitMs = 30000;

// The tile schedule of the handle's tuning (0 fields: the defaults) in its launch parameters.
void apply_tile_tuning(sssp_handle* h) {
  const sssp_tuning& t = h->tuning;
  h->p.inline_edges = t.inline_edges > 0 ? static_cast<uint32_t>(t.inline_edges) : kDefaultInlineEdges;
  h->p.hub_edges = t.hub_edges > 0 ? static_cast<uint32_t>(t.hub_edges) : sssp::kHub;
  h->p.chunk_entries = static_cast<uint32_t>(t.chunk_entries);
  h->chain = t.leader_chain == 1 || (t.leader_chain == 0 && h->m <= kChainMaxMeanDegree * h->n);
  // a chain runs the light steps of up to a full chunk of entries on the leader (the 4096 x 4096
  // grid: 3 % faster than a step of half a chunk, which is the default without chains)
  h->p.inline_entries = t.inline_entries > 0 ? static_cast<uint32_t>(t.inline_entries) : h->chain ? sssp::kChunk : 0u;
}

// A barrier wait that sees no progress for longer than this aborts the schedule (wall-clock ticks).
unsigned long long wait_ticks(const sssp_handle* h) {
  const int32_t ms = h->tuning.wait_limit_ms > 0 ? h->tuning.wait_limit_ms : kDefaultWaitLimitMs;
  return static_cast<unsigned long long>(ms) * static_cast<unsigned long long>(h->wallclock_khz);
}

sssp_status from_hip(hipError_t e) {
  if (e == hipSuccess) return SSSP_OK;
  if (e == hipErrorOutOfMemory) return SSSP_ERR_OUT_OF_MEMORY;
  return SSSP_ERR_DEVICE;
}

#define SSSP_TRY(expr)                           \
  do {                                           \
    sssp_status _st = from_hip(expr);            \
    if (_st != SSSP_OK) return _st;              \
  } while (0)

template <class T>
hipError_t dalloc(T** p, size_t count) {
  if (count == 0) count = 1;
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

void free_group(GroupMem& gm) {
  void* mem[] = {gm.tbuf[0], gm.tbuf[1], gm.texp, gm.qstamp, gm.sstamp, gm.bstamp, gm.fstamp, gm.ovf_at, gm.front[0],
                 gm.front[1], gm.slist, gm.bins, gm.far[0], gm.far[1], gm.hub};
  for (void* q : mem)
    if (q) (void)hipFree(q);
  gm = GroupMem{};
}

void free_adj_group(sssp_handle::AdjMem& am) {
  void* mem[] = {am.d, am.parent, am.cnt, am.lvl, am.g};
  for (void* q : mem)
    if (q) (void)hipFree(q);
  am = sssp_handle::AdjMem{};
}

// The first group's adjoint working set (all of it or none of it).
void free_adj(sssp_handle* h) {
  void* mem[] = {h->adj_d, h->adj_parent, h->adj_cnt, h->adj_lvl, h->adj_g, h->adj_grad64, h->adj_params_dev};
  for (void* q : mem)
    if (q) (void)hipFree(q);
  h->adj_d = nullptr;
  h->adj_parent = nullptr;
  h->adj_cnt = nullptr;
  h->adj_lvl = nullptr;
  h->adj_g = nullptr;
  h->adj_grad64 = nullptr;
  h->adj_params_dev = nullptr;
}

void free_handle(sssp_handle* h) {
  if (!h) return;
  sssp::Params& p = h->p;
  free_adj(h);
  void* extra[] = {h->inv, h->aux, h->params_dev, h->w64};
  for (void* q : extra)
    if (q) (void)hipFree(q);
  for (sssp_handle::AdjMem& am : h->adj_extra) free_adj_group(am);
  for (GroupMem& gm : h->extra) free_group(gm);
  void* dev[] = {h->off, h->split, const_cast<uint4*>(p.rows), const_cast<uint64_t*>(p.edges),
                 p.qstamp, p.sstamp, p.bstamp, p.fstamp, p.ovf_at, p.front[0], p.front[1], p.slist, p.bins,
                 p.far[0], p.far[1], p.hub, h->ctls, h->perm, h->src_dev, const_cast<uint32_t*>(p.vid), p.tbuf[0],
                 p.tbuf[1], p.texp};
  for (void* q : dev)
    if (q) (void)hipFree(q);
  if (h->src_host) (void)hipHostFree(h->src_host);
  if (h->ctl_host) (void)hipHostFree(h->ctl_host);
  if (h->aux_host) (void)hipHostFree(h->aux_host);
  delete h;
}

uint32_t pow2_at_least(uint32_t x) {
  uint32_t r = 1;
  while (r < x) r <<= 1;
  return r;
}

sssp_status configure_grid(sssp_handle* h) {
  if (h->occupancy < 1) return SSSP_ERR_UNSUPPORTED;
  h->grid = h->cus;
  h->grid_groups = h->occupancy_groups >= 2 ? 2 * h->cus : 0;
  return SSSP_OK;
}

// Whether a launch runs two 512-thread workgroups per CU (else one of 1024).
// The smaller workgroups are the default: measured faster on every workload
// (R-MAT scale 22 single source +2 %, scale 18 +6 %, the ragged batch +8 %,
// concurrent sources +15-20 %); workgroups_per_cu = 1 selects the larger ones
// for one source or one multi-source row.
bool small_workgroups(const sssp_handle* h, uint32_t groups, int multi) {
  (void)multi;
  if (h->grid_groups == 0) return false;
  return groups > 1 || h->tuning.workgroups_per_cu != 1;
}

// A weight (as bits) and delta as doubles (exact for every type).
double weight_of(const sssp_handle* h, uint64_t bits) {
  if (h->wtype == SSSP_WEIGHT_U32) return static_cast<double>(bits);
  if (h->wtype == SSSP_WEIGHT_F32) {
    float f;
    const uint32_t b = static_cast<uint32_t>(bits);
    std::memcpy(&f, &b, sizeof(f));
    return static_cast<double>(f);
  }
  double d;
  std::memcpy(&d, &bits, sizeof(d));
  return d;
}
double delta_of(const sssp_handle* h) {
  if (h->wtype == SSSP_WEIGHT_U32) return static_cast<double>(h->delta_u);
  if (h->wtype == SSSP_WEIGHT_F32) return static_cast<double>(h->delta_f);
  return h->delta_d;
}

sssp::Threshold threshold_of(const sssp_handle* h) {
  sssp::Threshold th{};
  th.wtype = h->wtype;
  th.delta_u = h->delta_u;
  th.delta_f = h->delta_f;
  th.delta_d = h->delta_d;
  return th;
}

// Floating-point bucket indices floor(t / delta) of every distance the solver
// can produce stay below 2^32 - 1 (the "none" tag). A tentative distance that
// wins an update is the rounded left-to-right sum along a simple path (a walk
// with a cycle never beats the value it had at the cycle's start), so it is
// at most the total weight times (1 + u)^(n-1), one rounding per edge (u =
// 2^-24 in fp32, 2^-53 in fp64). Integer distances fit by construction.
bool buckets_fit(const sssp_handle* h, double wsum) {
  if (h->wtype == SSSP_WEIGHT_U32) return true;
  const double u = h->wtype == SSSP_WEIGHT_F32 ? 0x1p-24 : 0x1p-53;
  const double bound = wsum * std::exp(static_cast<double>(h->n - 1) * u) * (1.0 + 0x1p-40);
  return bound / delta_of(h) < 4294967040.0;  // 2^32 - 256
}

// Every weight is light (w <= delta): A_H is empty.
uint32_t no_heavy_for(const sssp_handle* h, uint64_t wmax_bits) {
  return weight_of(h, wmax_bits) <= delta_of(h) ? 1u : 0u;
}

// Validation on the device: status bits, the largest weight (bits) and the
// weight total. With row_ptr == nullptr only the weights are checked.
struct WeightStats {
  uint32_t status;
  uint64_t wmax_bits;
  double wsum;
};
sssp_status validate_on_device(const int64_t* row_ptr, const int32_t* col, const void* w, int32_t wtype, int64_t n,
                               int64_t m, hipStream_t s, WeightStats* out) {
  uint32_t* scratch = nullptr;  // [0] status, [2..3] max weight bits, [4..5] fp64 weight total
  SSSP_TRY(dalloc(&scratch, 6));
  hipError_t e = hipMemsetAsync(scratch, 0, 6 * sizeof(uint32_t), s);
  auto* wmax = reinterpret_cast<unsigned long long*>(scratch + 2);
  auto* wsum = reinterpret_cast<double*>(scratch + 4);
  if (e == hipSuccess)
    e = row_ptr ? sssp::launch_validate(row_ptr, col, w, wtype, n, m, scratch, wmax, wsum, s)
                : sssp::launch_validate_weights(w, wtype, m, scratch, wmax, wsum, s);
  uint32_t res[6] = {0, 0, 0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(res, scratch, sizeof(res), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(scratch);
  SSSP_TRY(e);
  out->status = res[0];
  std::memcpy(&out->wmax_bits, res + 2, sizeof(uint64_t));
  std::memcpy(&out->wsum, res + 4, sizeof(double));
  return SSSP_OK;
}

// Working set of one more concurrent group: the same arrays as the first
// group's, with the de-duplication stamps cleared (its tags start at zero).
sssp_status alloc_group(sssp_handle* h, GroupMem* gm) {
  const size_t un = static_cast<size_t>(h->n);
  uint32_t** words[] = {&gm->qstamp, &gm->sstamp, &gm->bstamp, &gm->fstamp, &gm->ovf_at,
                        &gm->front[0], &gm->front[1], &gm->slist, &gm->far[0], &gm->far[1]};
  for (uint32_t** q : words) SSSP_TRY(dalloc(q, un));
  // distance words are 64-bit for every type (32-bit distances carry the frontier tag)
  for (void** q : {&gm->tbuf[0], &gm->tbuf[1]}) SSSP_TRY(hipMalloc(q, un * sizeof(uint64_t)));
  if (h->wtype == SSSP_WEIGHT_F64) SSSP_TRY(hipMalloc(&gm->texp, un * sizeof(uint64_t)));  // fp64 only
  SSSP_TRY(dalloc(&gm->bins, un * h->p.ring));
  SSSP_TRY(dalloc(&gm->hub, 2 * static_cast<size_t>(h->p.hub_cap)));
  uint32_t* zero[] = {gm->qstamp, gm->sstamp, gm->fstamp, gm->ovf_at};
  for (uint32_t* q : zero) SSSP_TRY(hipMemset(q, 0, un * sizeof(uint32_t)));
  return SSSP_OK;
}

// Write the per-group launch parameters to the device. Every group shares the
// graph and the schedule parameters; group g has its own control block and
// working set. Waits for the device first: a launch may still read them.
sssp_status upload_params(sssp_handle* h) {
  std::vector<sssp::Params> all(h->groups, h->p);
  for (uint32_t g = 0; g < h->groups; ++g) {
    sssp::Params& q = all[g];
    q.groups = h->groups;
    q.ctl = h->ctls + g;
    q.next_source = &h->ctls[0].next_source;
    if (g == 0) continue;
    const GroupMem& gm = h->extra[g - 1];
    q.tbuf[0] = gm.tbuf[0];
    q.tbuf[1] = gm.tbuf[1];
    q.texp = gm.texp;
    q.qstamp = gm.qstamp;
    q.sstamp = gm.sstamp;
    q.bstamp = gm.bstamp;
    q.fstamp = gm.fstamp;
    q.ovf_at = gm.ovf_at;
    q.front[0] = gm.front[0];
    q.front[1] = gm.front[1];
    q.slist = gm.slist;
    q.bins = gm.bins;
    q.far[0] = gm.far[0];
    q.far[1] = gm.far[1];
    q.hub = gm.hub;
  }
  sssp::Params single = h->p;  // the whole grid as one group (multi-source solves)
  single.groups = 1;
  single.ctl = h->ctls;
  single.next_source = &h->ctls[0].next_source;
  SSSP_TRY(hipDeviceSynchronize());
  SSSP_TRY(hipMemcpy(h->params_dev, all.data(), sizeof(sssp::Params) * all.size(), hipMemcpyHostToDevice));
  SSSP_TRY(hipMemcpy(h->params_dev + sssp::kMaxGroups, &single, sizeof(single), hipMemcpyHostToDevice));
  return SSSP_OK;
}

// Clear the de-duplication stamps and overflow marks of the groups of the next
// launch with fill kernels (no memset nodes when the stream is being captured).
sssp_status clear_stamps(sssp_handle* h, hipStream_t s) {
  const size_t un = static_cast<size_t>(h->n);
  for (uint32_t g = 0; g < h->groups; ++g) {
    uint32_t* q[4];
    if (g == 0) {
      q[0] = h->p.qstamp, q[1] = h->p.sstamp, q[2] = h->p.fstamp, q[3] = h->p.ovf_at;
    } else {
      const GroupMem& gm = h->extra[g - 1];
      q[0] = gm.qstamp, q[1] = gm.sstamp, q[2] = gm.fstamp, q[3] = gm.ovf_at;
    }
    for (uint32_t* a : q) SSSP_TRY(sssp::launch_fill(a, un, 0u, s));
  }
  return SSSP_OK;
}

sssp_status create_impl(const sssp_graph* g, double delta, hipStream_t stream, sssp_handle* h) {
  SSSP_TRY(hipGetDevice(&h->device));
  if (scratch_address(h->device, &h->scratch) != hipSuccess) h->scratch = nullptr;
  hipDeviceProp_t prop;
  SSSP_TRY(hipGetDeviceProperties(&prop, h->device));
  if (!prop.cooperativeLaunch) return SSSP_ERR_UNSUPPORTED;
  h->cus = prop.multiProcessorCount;
  {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device) == hipSuccess && khz > 0)
      h->wallclock_khz = khz;
  }
  {  // both solver kernels (with and without chained steps) must fit the grid
    int occ[4] = {0, 0, 0, 0};
    SSSP_TRY(sssp::solver_occupancy(g->wtype, sssp::kWG, false, &occ[0]));
    SSSP_TRY(sssp::solver_occupancy(g->wtype, sssp::kWG, true, &occ[1]));
    SSSP_TRY(sssp::solver_occupancy(g->wtype, sssp::kWGGroups, false, &occ[2]));
    SSSP_TRY(sssp::solver_occupancy(g->wtype, sssp::kWGGroups, true, &occ[3]));
    h->occupancy = std::min(occ[0], occ[1]);
    h->occupancy_groups = std::min(occ[2], occ[3]);
  }

  const int64_t n = g->n, m = g->m;
  h->n = n;
  h->m = m;
  h->wtype = g->wtype;
  h->delta = delta;
  if (g->wtype == SSSP_WEIGHT_U32) h->delta_u = static_cast<uint32_t>(delta);
  else if (g->wtype == SSSP_WEIGHT_F32) h->delta_f = static_cast<float>(delta);
  else h->delta_d = delta;

  // 1. validate the CSR and the weights on the device
  WeightStats ws{};
  const sssp_status vs = validate_on_device(g->row_ptr, g->col_idx, g->weights, g->wtype, n, m, stream, &ws);
  if (vs != SSSP_OK) return vs;
  if (ws.status & (sssp::kBadRowPtr | sssp::kBadCol)) return SSSP_ERR_INVALID_ARGUMENT;
  if (ws.status & sssp::kBadWeight) return SSSP_ERR_INVALID_WEIGHT;
  h->wmax_bits = ws.wmax_bits;

  // 2. bucket geometry: ring large enough that one relaxation never jumps past it
  const double span = weight_of(h, h->wmax_bits) / delta_of(h);  // max weight / delta
  if (!buckets_fit(h, ws.wsum)) return SSSP_ERR_UNSUPPORTED;
  uint32_t ring = h->tuning.ring_buckets > 0 ? static_cast<uint32_t>(h->tuning.ring_buckets)
                                              : pow2_at_least(static_cast<uint32_t>(std::min(span + 2.0, 64.0)));
  if (ring < 2) ring = 2;
  if (ring > sssp::kRingMax || (ring & (ring - 1))) return SSSP_ERR_INVALID_ARGUMENT;

  // 3. device memory
  sssp::Params& p = h->p;
  p.n = static_cast<uint32_t>(n);
  p.ring = ring;
  p.ring_mask = ring - 1;
  p.wtype = static_cast<uint32_t>(g->wtype);
  p.no_heavy = no_heavy_for(h, h->wmax_bits);
  p.delta_u = h->delta_u;
  p.delta_d = g->wtype == SSSP_WEIGHT_U32 ? 0.0 : delta_of(h);
  p.inv_delta_d = p.delta_d > 0 ? 1.0 / p.delta_d : 0.0;
  const size_t un = static_cast<size_t>(n), um = static_cast<size_t>(m);
  uint32_t *off = nullptr, *split = nullptr;
  uint64_t* edges = nullptr;
  SSSP_TRY(dalloc(&off, un + 1));
  h->off = off;
  SSSP_TRY(dalloc(&split, un));
  h->split = split;
  uint4* rows = nullptr;
  SSSP_TRY(dalloc(&rows, un));
  p.rows = rows;
  SSSP_TRY(dalloc(&edges, um));
  p.edges = edges;
  SSSP_TRY(dalloc(&h->perm, um));
  SSSP_TRY(dalloc(&p.qstamp, un));
  SSSP_TRY(dalloc(&p.sstamp, un));
  SSSP_TRY(dalloc(&p.bstamp, un));
  SSSP_TRY(dalloc(&p.fstamp, un));
  SSSP_TRY(dalloc(&p.ovf_at, un));
  // each vertex appears at most once in a phase's list, so the pieces of its high-degree
  // vertices number at most m / kPieceMin + m / kHubMin (pieces of the smaller workgroup,
  // the smallest hub threshold a tuning may set)
  p.hub_cap = static_cast<uint32_t>(um / sssp::kPieceMin + um / sssp::kHubMin + 16);
  SSSP_TRY(dalloc(&p.hub, 2 * static_cast<size_t>(p.hub_cap)));
  apply_tile_tuning(h);
  SSSP_TRY(dalloc(&p.front[0], un));
  SSSP_TRY(dalloc(&p.front[1], un));
  SSSP_TRY(dalloc(&p.slist, un));
  SSSP_TRY(dalloc(&p.bins, un * ring));
  SSSP_TRY(dalloc(&p.far[0], un));
  SSSP_TRY(dalloc(&p.far[1], un));
  SSSP_TRY(dalloc(&h->ctls, sssp::kMaxGroups));
  p.ctl = h->ctls;
  p.next_source = &h->ctls[0].next_source;
  p.groups = 1;
  SSSP_TRY(dalloc(&h->params_dev, sssp::kMaxGroups + 1));
  SSSP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->ctl_host), sizeof(sssp::Ctl) * sssp::kMaxGroups,
                         hipHostMallocDefault));
  SSSP_TRY(hipMemsetAsync(p.qstamp, 0, un * sizeof(uint32_t), stream));
  SSSP_TRY(hipMemsetAsync(p.sstamp, 0, un * sizeof(uint32_t), stream));
  SSSP_TRY(hipMemsetAsync(p.fstamp, 0, un * sizeof(uint32_t), stream));
  SSSP_TRY(hipMemsetAsync(p.ovf_at, 0, un * sizeof(uint32_t), stream));
  SSSP_TRY(hipMemsetAsync(h->ctls, 0, sizeof(sssp::Ctl) * sssp::kMaxGroups, stream));
  SSSP_TRY(sssp::launch_ctl_reset(h->ctls, sssp::kMaxGroups, 1, nullptr, 0, wait_ticks(h), stream));

  // 4. relabel by in-degree, then the light/heavy split (A_L, A_H)
  uint32_t* vid = nullptr;
  SSSP_TRY(dalloc(&vid, un));
  p.vid = vid;
  SSSP_TRY(hipMalloc(&p.tbuf[0], un * sizeof(uint64_t)));  // 64-bit distance words (see the kernels)
  SSSP_TRY(hipMalloc(&p.tbuf[1], un * sizeof(uint64_t)));
  if (g->wtype == SSSP_WEIGHT_F64) SSSP_TRY(hipMalloc(&p.texp, un * sizeof(uint64_t)));  // fp64 only
  if (g->wtype == SSSP_WEIGHT_F64) SSSP_TRY(dalloc(&h->w64, um));
  p.w64 = h->w64;
  uint32_t* build = nullptr;
  SSSP_TRY(dalloc(&build, sssp::build_scratch_words(n)));
  hipError_t be = sssp::launch_relabel_and_split(g->row_ptr, g->col_idx, g->weights, threshold_of(h), n, m, build, vid,
                                                 off, split, edges, h->w64, h->perm, stream);
  if (be == hipSuccess) be = sssp::launch_pack_rows(off, split, n, rows, stream);
  if (be == hipSuccess) be = dalloc(&h->inv, un);
  if (be == hipSuccess) be = sssp::launch_inverse(vid, n, h->inv, stream);
  if (be == hipSuccess) be = dalloc(&h->aux, 2);
  if (be == hipSuccess)
    be = hipHostMalloc(reinterpret_cast<void**>(&h->aux_host), 2 * sizeof(unsigned long long), hipHostMallocDefault);
  if (be == hipSuccess) {
    int occ = 0;
    be = sssp::adjoint_occupancy(&occ);
    h->adj_grid = occ >= 1 ? h->cus : 0;
  }
  if (be == hipSuccess) be = hipStreamSynchronize(stream);
  uint32_t no_in_edges = 0;
  if (be == hipSuccess)
    be = hipMemcpy(&no_in_edges, build + sssp::relabel_no_in_edges_word(n), sizeof(uint32_t), hipMemcpyDeviceToHost);
  p.zero_from = static_cast<uint32_t>(n) - (no_in_edges <= static_cast<uint32_t>(n) ? no_in_edges : 0u);
  (void)hipFree(build);
  SSSP_TRY(be);
  const sssp_status st = configure_grid(h);
  if (st != SSSP_OK) return st;
  return upload_params(h);
}

// Copy host sources into the handle's device buffer (checked against n).
sssp_status stage_sources(sssp_handle* h, const int32_t* sources, int32_t k, hipStream_t s) {
  for (int32_t r = 0; r < k; ++r)
    if (sources[r] < 0 || sources[r] >= h->n) return SSSP_ERR_INVALID_ARGUMENT;
  if (k > h->src_cap) {
    if (h->src_dev) (void)hipFree(h->src_dev);
    if (h->src_host) (void)hipHostFree(h->src_host);
    h->src_dev = nullptr;
    h->src_host = nullptr;
    h->src_cap = 0;
    SSSP_TRY(dalloc(&h->src_dev, static_cast<size_t>(k)));
    SSSP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->src_host), sizeof(int32_t) * k, hipHostMallocDefault));
    h->src_cap = k;
  }
  SSSP_TRY(hipStreamSynchronize(s));  // the pinned staging buffer may still feed an earlier copy
  std::memcpy(h->src_host, sources, sizeof(int32_t) * k);
  SSSP_TRY(hipMemcpyAsync(h->src_dev, h->src_host, sizeof(int32_t) * k, hipMemcpyHostToDevice, s));
  return SSSP_OK;
}

// ring-size rule of set_weights (as in create)
uint32_t ring_for(const sssp_handle* h, uint64_t wmax_bits) {
  const double span = weight_of(h, wmax_bits) / delta_of(h);
  uint32_t ring = pow2_at_least(static_cast<uint32_t>(std::min(span + 2.0, 64.0)));
  return ring < 2 ? 2 : ring;
}

// Enqueue one solver launch over k sources read from device memory: a reset of
// the groups' control blocks (a kernel), then the cooperative launch.
sssp_status enqueue_solve(sssp_handle* h, const int32_t* sources_dev, int32_t k, int multi, void* dist,
                          hipStream_t s) {
  const uint32_t groups = multi ? 1u : h->groups;
  int reset_epochs = 0;
  if (h->stamps_dirty) {  // an aborted launch may have left stamps and marks behind
    const sssp_status st = clear_stamps(h, s);
    if (st != SSSP_OK) return st;
    reset_epochs = 1;
    h->stamps_dirty = false;
  }
  SSSP_TRY(sssp::launch_ctl_reset(h->ctls, groups, reset_epochs, h->trace, h->trace_cap, wait_ticks(h), s));
  // concurrent sources run on two smaller workgroups per CU; one source (or one
  // multi-source row) on one full workgroup per CU
  const bool small = small_workgroups(h, groups, multi);
  SSSP_TRY(sssp::launch_solver(multi ? h->params_dev + sssp::kMaxGroups : h->params_dev, groups, h->p.wtype,
                               sources_dev, k, multi, static_cast<uint32_t*>(dist), small ? h->grid_groups : h->grid,
                               small ? sssp::kWGGroups : sssp::kWG, h->chain, s));
  h->enq_groups = groups;
  return SSSP_OK;
}

// Wait for the last enqueued launch and turn its control blocks into a status
// and the statistics of sssp_last_stats.
sssp_status read_status(sssp_handle* h, hipStream_t s) {
  if (h->enq_groups == 0) return SSSP_ERR_NO_FORWARD;
  const uint32_t groups = h->enq_groups;
  SSSP_TRY(hipMemcpyAsync(h->ctl_host, h->ctls, sizeof(sssp::Ctl) * groups, hipMemcpyDeviceToHost, s));
  SSSP_TRY(hipStreamSynchronize(s));
  sssp_stats st{};
  bool abort = false, ovf = false, bad = false;
  for (uint32_t g = 0; g < groups; ++g) {
    const sssp::Ctl& c = h->ctl_host[g];
    abort |= c.abort != 0;
    ovf |= c.ovf_real != 0;
    bad |= c.bad_source != 0;
    st.sources += c.sources;
    st.buckets += c.buckets;
    st.light_phases += c.light_phases;
    st.heavy_phases += c.heavy_phases;
    st.far_phases += c.far_phases;
    st.light_edges += c.light_edges;
    st.heavy_edges += c.heavy_edges;
    st.improvements += c.improvements;
    st.attempts += c.attempts;
    st.barriers += c.barriers;
    st.trace_records += c.trace_len;
  }
  if (abort) {
    h->stamps_dirty = true;
    return SSSP_ERR_DEVICE;
  }
  h->last = st;
  if (bad) return SSSP_ERR_INVALID_ARGUMENT;
  if (ovf) return SSSP_ERR_OVERFLOW;
  h->solved = true;
  return SSSP_OK;
}

// Launch the adjoint over `groups` groups whose working sets are already in
// h->adj_host (d, parent, cnt, lvl, g) and read its outcome. params_dev: device
// room for the groups' launch parameters; grad64: the fp64 dL/dw accumulator
// [m]; sources: DEVICE [k] (checked on the device). Allocates nothing.
sssp_status run_adjoint(sssp_handle* h, uint32_t groups, sssp::AdjParams* params_dev, double* grad64,
                        const int32_t* sources, int32_t k, const void* dist, const float* grad_dist, float* grad_w,
                        hipStream_t s) {
  for (uint32_t gi = 0; gi < groups; ++gi) {
    sssp::AdjParams& a = h->adj_host[gi];
    a.n = static_cast<uint32_t>(h->n);
    a.m = static_cast<uint64_t>(h->m);
    a.vid = h->p.vid;
    a.inv = h->inv;
    a.rows = h->p.rows;
    a.edges = h->p.edges;
    a.perm = h->perm;
    a.grad64 = grad64;
    a.ctl = h->ctls + gi;
    a.next_source = &h->ctls[0].next_source;
    // the level lists reuse the frontier buffers of the group's solver working set
    a.front[0] = gi == 0 ? h->p.front[0] : h->extra[gi - 1].front[0];
    a.front[1] = gi == 0 ? h->p.front[1] : h->extra[gi - 1].front[1];
  }
  SSSP_TRY(hipMemcpyAsync(params_dev, h->adj_host, sizeof(sssp::AdjParams) * groups, hipMemcpyHostToDevice, s));
  SSSP_TRY(sssp::launch_fill(reinterpret_cast<uint32_t*>(h->aux), 4, 0u, s));
  SSSP_TRY(sssp::launch_count_reached(static_cast<const uint32_t*>(dist), static_cast<uint32_t>(h->n), k, h->wtype,
                                      h->aux, s));
  SSSP_TRY(sssp::launch_ctl_reset(h->ctls, groups, 0, nullptr, 0, wait_ticks(h), s));
  SSSP_TRY(sssp::launch_adjoint(params_dev, groups, sources, k, static_cast<const uint32_t*>(dist), grad_dist, grad_w,
                                static_cast<uint64_t>(h->m), grad64, h->adj_grid, s));
  SSSP_TRY(hipMemcpyAsync(h->ctl_host, h->ctls, sizeof(sssp::Ctl) * groups, hipMemcpyDeviceToHost, s));
  SSSP_TRY(hipMemcpyAsync(h->aux_host, h->aux, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  SSSP_TRY(hipStreamSynchronize(s));
  const unsigned long long reached = *h->aux_host;
  bool abort = false, bad = false, bad_source = false;
  unsigned long long released = 0;
  for (uint32_t gi = 0; gi < groups; ++gi) {
    const sssp::Ctl& c = h->ctl_host[gi];
    abort |= c.abort != 0;
    bad |= c.ovf_real != 0;
    bad_source |= c.bad_source != 0;
    released += c.adj_released;
  }
  if (abort) return SSSP_ERR_DEVICE;
  if (bad_source) return SSSP_ERR_INVALID_ARGUMENT;
  // an infeasible edge, a reached vertex without a tight in-edge, d(s) != 0, or parents that never lead to s
  if (bad || released != reached) return SSSP_ERR_INVALID_ARGUMENT;
  return SSSP_OK;
}

}  // namespace

extern "C" {

const char* sssp_status_string(sssp_status s) {
  switch (s) {
    case SSSP_OK: return "ok";
    case SSSP_ERR_INVALID_ARGUMENT: return "invalid argument";
    case SSSP_ERR_INVALID_WEIGHT: return "invalid weight";
    case SSSP_ERR_OUT_OF_MEMORY: return "out of device memory";
    case SSSP_ERR_DEVICE: return "device error";
    case SSSP_ERR_OVERFLOW: return "distance overflow";
    case SSSP_ERR_NO_FORWARD: return "no forward solve";
    case SSSP_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

sssp_status sssp_create(const sssp_graph* g, double delta, void* stream, sssp_handle** out) {
  if (!out) return SSSP_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!g || !g->row_ptr) return SSSP_ERR_INVALID_ARGUMENT;
  if (g->wtype != SSSP_WEIGHT_U32 && g->wtype != SSSP_WEIGHT_F32 && g->wtype != SSSP_WEIGHT_F64)
    return SSSP_ERR_INVALID_ARGUMENT;
  if (g->n < 1 || g->m < 0) return SSSP_ERR_INVALID_ARGUMENT;
  if (g->n >= (int64_t(1) << 31) || g->m >= (int64_t(1) << 32) - 1) return SSSP_ERR_UNSUPPORTED;
  if (g->m > 0 && (!g->col_idx || !g->weights)) return SSSP_ERR_INVALID_ARGUMENT;
  if (!std::isfinite(delta) || !(delta > 0)) return SSSP_ERR_INVALID_ARGUMENT;
  if (g->wtype == SSSP_WEIGHT_U32) {
    if (delta != std::floor(delta) || delta < 1.0 || delta > 4294967295.0) return SSSP_ERR_INVALID_ARGUMENT;
  } else if (g->wtype == SSSP_WEIGHT_F32) {
    const float df = static_cast<float>(delta);
    if (!std::isfinite(df) || !(df > 0.0f)) return SSSP_ERR_INVALID_ARGUMENT;
  }
  sssp_handle* h = new (std::nothrow) sssp_handle();
  if (!h) return SSSP_ERR_OUT_OF_MEMORY;
  const sssp_status st = create_impl(g, delta, static_cast<hipStream_t>(stream), h);
  if (st != SSSP_OK) {
    (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
    free_handle(h);
    return st;
  }
  *out = h;
  return SSSP_OK;
}

sssp_status sssp_solve(sssp_handle* h, const int32_t* sources, int32_t k, void* dist, void* stream) {
  if (!h || !sources || k < 1 || !dist) return SSSP_ERR_INVALID_ARGUMENT;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SSSP_TRY(hipSetDevice(h->device));
  sssp_status st = stage_sources(h, sources, k, s);
  if (st == SSSP_OK) st = enqueue_solve(h, h->src_dev, k, 0, dist, s);
  if (st != SSSP_OK) return st;
  return read_status(h, s);
}

sssp_status sssp_solve_async(sssp_handle* h, const int32_t* sources, int32_t k, void* dist, void* stream) {
  if (!h || !sources || k < 1 || !dist) return SSSP_ERR_INVALID_ARGUMENT;
  SSSP_TRY(hipSetDevice(h->device));
  return enqueue_solve(h, sources, k, 0, dist, static_cast<hipStream_t>(stream));
}

sssp_status sssp_solve_multi(sssp_handle* h, const int32_t* sources, int32_t k, void* dist, void* stream) {
  if (!h || !sources || k < 1 || !dist) return SSSP_ERR_INVALID_ARGUMENT;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SSSP_TRY(hipSetDevice(h->device));
  sssp_status st = stage_sources(h, sources, k, s);
  if (st == SSSP_OK) st = enqueue_solve(h, h->src_dev, k, 1, dist, s);
  if (st != SSSP_OK) return st;
  return read_status(h, s);
}

sssp_status sssp_solve_multi_async(sssp_handle* h, const int32_t* sources, int32_t k, void* dist, void* stream) {
  if (!h || !sources || k < 1 || !dist) return SSSP_ERR_INVALID_ARGUMENT;
  SSSP_TRY(hipSetDevice(h->device));
  return enqueue_solve(h, sources, k, 1, dist, static_cast<hipStream_t>(stream));
}

sssp_status sssp_solve_status(sssp_handle* h, void* stream) {
  if (!h) return SSSP_ERR_INVALID_ARGUMENT;
  SSSP_TRY(hipSetDevice(h->device));
  return read_status(h, static_cast<hipStream_t>(stream));
}

sssp_status sssp_backward(sssp_handle* h, const int32_t* sources, int32_t k, const void* dist,
                          const float* grad_dist, float* grad_w, void* stream) {
  if (!h || !sources || k < 1 || !dist || !grad_dist || !grad_w) return SSSP_ERR_INVALID_ARGUMENT;
  if (h->wtype != SSSP_WEIGHT_F32 || h->adj_grid < 1) return SSSP_ERR_UNSUPPORTED;
  if (!h->solved) return SSSP_ERR_NO_FORWARD;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SSSP_TRY(hipSetDevice(h->device));
  const size_t un = static_cast<size_t>(h->n), um = static_cast<size_t>(h->m);
  if (!h->adj_d) {  // allocated whole or not at all (a later call tests adj_d only)
    hipError_t e = dalloc(&h->adj_d, un);
    if (e == hipSuccess) e = dalloc(&h->adj_parent, un);
    if (e == hipSuccess) e = dalloc(&h->adj_cnt, un);
    if (e == hipSuccess) e = dalloc(&h->adj_lvl, un);
    if (e == hipSuccess) e = dalloc(&h->adj_g, un);
    if (e == hipSuccess) e = dalloc(&h->adj_grad64, um);
    if (e == hipSuccess) e = dalloc(&h->adj_params_dev, sssp::kMaxGroups);
    if (e != hipSuccess) {
      free_adj(h);
      return from_hip(e);
    }
  }
  // sources share the launch as in the forward solve: one group per concurrent source
  const uint32_t groups = h->adj_grid % static_cast<int>(h->groups) == 0 ? h->groups : 1u;
  while (h->adj_extra.size() + 1 < groups) {
    h->adj_extra.emplace_back();
    sssp_handle::AdjMem& am = h->adj_extra.back();
    hipError_t e = dalloc(&am.d, un);
    if (e == hipSuccess) e = dalloc(&am.parent, un);
    if (e == hipSuccess) e = dalloc(&am.cnt, un);
    if (e == hipSuccess) e = dalloc(&am.lvl, un);
    if (e == hipSuccess) e = dalloc(&am.g, un);
    if (e != hipSuccess) {  // a partly allocated working set is not kept
      free_adj_group(am);
      h->adj_extra.pop_back();
      return from_hip(e);
    }
  }
  const sssp_status st = stage_sources(h, sources, k, s);
  if (st != SSSP_OK) return st;
  for (uint32_t gi = 0; gi < groups; ++gi) {
    sssp::AdjParams& a = h->adj_host[gi];
    if (gi == 0) {
      a.d = h->adj_d;
      a.parent = h->adj_parent;
      a.cnt = h->adj_cnt;
      a.lvl = h->adj_lvl;
      a.g = h->adj_g;
    } else {
      const sssp_handle::AdjMem& am = h->adj_extra[gi - 1];
      a.d = am.d;
      a.parent = am.parent;
      a.cnt = am.cnt;
      a.lvl = am.lvl;
      a.g = am.g;
    }
  }
  return run_adjoint(h, groups, h->adj_params_dev, h->adj_grad64, h->src_dev, k, dist, grad_dist, grad_w, s);
}

sssp_status sssp_backward_noalloc(sssp_handle* h, const int32_t* sources, int32_t k, const void* dist,
                                  const float* grad_dist, float* grad_w, void* stream) {
  if (!h || !sources || k < 1 || !dist || !grad_dist || !grad_w) return SSSP_ERR_INVALID_ARGUMENT;
  if (h->wtype != SSSP_WEIGHT_F32 || h->adj_grid < 1) return SSSP_ERR_UNSUPPORTED;
  if (!h->solved) return SSSP_ERR_NO_FORWARD;
  if (!h->scratch) return SSSP_ERR_DEVICE;  // the array's address could not be resolved at create
  hipStream_t s = static_cast<hipStream_t>(stream);
  SSSP_TRY(hipSetDevice(h->device));
  // carve the scratch array: launch parameters, dL/dw accumulator, then one working set per group
  const size_t un = static_cast<size_t>(h->n), um = static_cast<size_t>(h->m);
  static_assert(sizeof(sssp::AdjParams) * sssp::kMaxGroups <= 35 * 1024, "the header states 34 KiB");
  const size_t params_bytes = align256(sizeof(sssp::AdjParams) * sssp::kMaxGroups);
  const size_t grad_bytes = align256(um * sizeof(double));
  const size_t group_bytes = align256(un * sizeof(uint32_t)) * 3 + align256(un * sizeof(unsigned long long)) +
                             align256(un * sizeof(double));
  if (params_bytes + grad_bytes + group_bytes > kNoAllocScratchBytes) return SSSP_ERR_UNSUPPORTED;
  const size_t fit = (kNoAllocScratchBytes - params_bytes - grad_bytes) / group_bytes;
  // as many concurrent groups as the forward solve uses, if they fit (a divisor of the grid), else fewer
  uint32_t groups = h->adj_grid % static_cast<int>(h->groups) == 0 ? h->groups : 1u;
  while (groups > 1 && groups > fit) groups >>= 1;
  while (groups > 1 && h->adj_grid % static_cast<int>(groups) != 0) groups >>= 1;
  char* base = static_cast<char*>(h->scratch);
  auto* params_dev = reinterpret_cast<sssp::AdjParams*>(base);
  auto* grad64 = reinterpret_cast<double*>(base + params_bytes);
  char* at = base + params_bytes + grad_bytes;
  for (uint32_t gi = 0; gi < groups; ++gi) {
    sssp::AdjParams& a = h->adj_host[gi];
    a.d = reinterpret_cast<uint32_t*>(at);
    at += align256(un * sizeof(uint32_t));
    a.cnt = reinterpret_cast<uint32_t*>(at);
    at += align256(un * sizeof(uint32_t));
    a.lvl = reinterpret_cast<uint32_t*>(at);
    at += align256(un * sizeof(uint32_t));
    a.parent = reinterpret_cast<unsigned long long*>(at);
    at += align256(un * sizeof(unsigned long long));
    a.g = reinterpret_cast<double*>(at);
    at += align256(un * sizeof(double));
  }
  return run_adjoint(h, groups, params_dev, grad64, sources, k, dist, grad_dist, grad_w, s);
}

sssp_status sssp_set_weights(sssp_handle* h, const void* weights, void* stream) {
  if (!h || (h->m > 0 && !weights)) return SSSP_ERR_INVALID_ARGUMENT;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SSSP_TRY(hipSetDevice(h->device));
  if (h->m == 0) return SSSP_OK;
  WeightStats ws{};
  const sssp_status vs = validate_on_device(nullptr, nullptr, weights, h->wtype, h->n, h->m, s, &ws);
  if (vs != SSSP_OK) return vs;
  if (ws.status & sssp::kBadWeight) return SSSP_ERR_INVALID_WEIGHT;
  if (!buckets_fit(h, ws.wsum)) return SSSP_ERR_UNSUPPORTED;
  sssp::Params& p = h->p;
  const size_t un = static_cast<size_t>(h->n), um = static_cast<size_t>(h->m);
  const uint32_t ring = ring_for(h, ws.wmax_bits);
  if (ring > p.ring) {  // a larger weight spread needs more near buckets (in every group)
    SSSP_TRY(hipDeviceSynchronize());
    // all the larger rings first: on a failure the handle keeps its old ones
    std::vector<uint32_t*> bins(h->extra.size() + 1, nullptr);
    hipError_t e = hipSuccess;
    for (uint32_t*& b : bins)
      if (e == hipSuccess) e = dalloc(&b, un * ring);
    if (e != hipSuccess) {
      for (uint32_t* b : bins)
        if (b) (void)hipFree(b);
      return from_hip(e);
    }
    (void)hipFree(p.bins);
    p.bins = bins[0];
    for (size_t g = 0; g < h->extra.size(); ++g) {
      (void)hipFree(h->extra[g].bins);
      h->extra[g].bins = bins[g + 1];
    }
    p.ring = ring;
    p.ring_mask = ring - 1;
  }
  uint4* rows = nullptr;
  uint64_t* edges = nullptr;
  uint32_t* perm = nullptr;
  uint64_t* w64 = nullptr;
  hipError_t e = dalloc(&rows, un);
  if (e == hipSuccess) e = dalloc(&edges, um);
  if (e == hipSuccess) e = dalloc(&perm, um);
  if (e == hipSuccess && h->wtype == SSSP_WEIGHT_F64) e = dalloc(&w64, um);
  if (e == hipSuccess)
    e = sssp::launch_resplit(static_cast<uint32_t>(h->n), p.rows, p.edges, h->perm, weights, threshold_of(h), rows,
                             w64, edges, perm, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    void* mem[] = {rows, edges, perm, w64};
    for (void* q : mem)
      if (q) (void)hipFree(q);
    return from_hip(e);
  }
  (void)hipFree(const_cast<uint4*>(p.rows));
  (void)hipFree(const_cast<uint64_t*>(p.edges));
  (void)hipFree(h->perm);
  if (h->w64) (void)hipFree(h->w64);
  p.rows = rows;
  p.edges = edges;
  p.w64 = w64;
  h->w64 = w64;
  h->perm = perm;
  h->wmax_bits = ws.wmax_bits;
  p.no_heavy = no_heavy_for(h, h->wmax_bits);
  h->solved = false;  // distances of earlier solves used the old weights
  return upload_params(h);
}

sssp_status sssp_last_stats(const sssp_handle* h, sssp_stats* out) {
  if (!h || !out) return SSSP_ERR_INVALID_ARGUMENT;
  *out = h->last;
  return SSSP_OK;
}

sssp_status sssp_set_tuning(sssp_handle* h, const sssp_tuning* t) {
  if (!h || !t) return SSSP_ERR_INVALID_ARGUMENT;
  if (t->workgroups_per_cu < 0 || t->ring_buckets < 0 || t->inline_edges < 0 || t->concurrent_sources < 0 ||
      t->wait_limit_ms < 0 || t->hub_edges < 0 || t->chunk_entries < 0 || t->inline_entries < 0 ||
      t->leader_chain < 0 || t->leader_chain > 2)
    return SSSP_ERR_INVALID_ARGUMENT;
  const auto pow2 = [](int32_t x) { return (x & (x - 1)) == 0; };
  if (t->hub_edges != 0 && (t->hub_edges < static_cast<int32_t>(sssp::kHubMin) || t->hub_edges > 65536 ||
                            !pow2(t->hub_edges)))
    return SSSP_ERR_INVALID_ARGUMENT;
  if (t->chunk_entries != 0 && (t->chunk_entries < static_cast<int32_t>(sssp::kMinChunk) ||
                                t->chunk_entries > static_cast<int32_t>(sssp::kChunk) || !pow2(t->chunk_entries)))
    return SSSP_ERR_INVALID_ARGUMENT;
  if (t->inline_entries > static_cast<int32_t>(sssp::kChunk)) return SSSP_ERR_INVALID_ARGUMENT;
  if (t->ring_buckets != 0 && t->ring_buckets != static_cast<int32_t>(h->p.ring))
    return SSSP_ERR_UNSUPPORTED;  // the ring is sized at create time
  SSSP_TRY(hipSetDevice(h->device));
  const sssp_tuning old = h->tuning;
  const int old_grid = h->grid, old_grid_groups = h->grid_groups;
  h->tuning = *t;
  sssp_status st = configure_grid(h);
  const uint32_t groups = t->concurrent_sources > 0 ? static_cast<uint32_t>(t->concurrent_sources) : 1u;
  if (st == SSSP_OK && (groups > sssp::kMaxGroups || h->grid % static_cast<int>(groups) != 0 ||
                        h->grid_groups % static_cast<int>(groups) != 0))
    st = SSSP_ERR_UNSUPPORTED;  // every group gets the same number of workgroups
  while (st == SSSP_OK && h->extra.size() + 1 < groups) {
    h->extra.emplace_back();
    st = alloc_group(h, &h->extra.back());
    if (st != SSSP_OK) {  // a partly allocated working set is not kept
      free_group(h->extra.back());
      h->extra.pop_back();
    }
  }
  if (st != SSSP_OK) {
    h->tuning = old;
    h->grid = old_grid;
    h->grid_groups = old_grid_groups;
    return st;
  }
  h->groups = groups;
  apply_tile_tuning(h);
  return upload_params(h);
}

sssp_status sssp_get_tuning(const sssp_handle* h, sssp_tuning* out) {
  if (!h || !out) return SSSP_ERR_INVALID_ARGUMENT;
  sssp_tuning t{};
  const uint32_t groups = h->groups;
  const bool small = small_workgroups(h, groups, 0);
  const uint32_t size = static_cast<uint32_t>(small ? h->grid_groups : h->grid) / groups;
  t.workgroups_per_cu = small ? 2 : 1;
  t.ring_buckets = static_cast<int32_t>(h->p.ring);
  t.inline_edges = static_cast<int32_t>(h->p.inline_edges);
  t.concurrent_sources = static_cast<int32_t>(groups);
  t.wait_limit_ms = h->tuning.wait_limit_ms > 0 ? h->tuning.wait_limit_ms : kDefaultWaitLimitMs;
  t.hub_edges = static_cast<int32_t>(h->p.hub_edges);
  const uint32_t chunk = h->p.chunk_entries ? h->p.chunk_entries : (size >= 128 ? sssp::kChunk / 2 : sssp::kChunk);
  t.chunk_entries = static_cast<int32_t>(chunk);
  t.inline_entries = static_cast<int32_t>(h->p.inline_entries ? h->p.inline_entries : chunk);
  t.leader_chain = h->chain ? 1 : 2;
  *out = t;
  return SSSP_OK;
}

sssp_status sssp_set_trace(sssp_handle* h, uint64_t* device_buffer, int64_t capacity) {
  if (!h || capacity < 0 || (capacity > 0 && !device_buffer)) return SSSP_ERR_INVALID_ARGUMENT;
  if (capacity > 0xFFFFFFFFll) capacity = 0xFFFFFFFFll;
  h->trace = capacity > 0 ? reinterpret_cast<unsigned long long*>(device_buffer) : nullptr;
  h->trace_cap = static_cast<uint32_t>(capacity);
  return SSSP_OK;
}

sssp_status sssp_graph_info(const sssp_handle* h, int64_t* n, int64_t* m, int32_t* wtype) {
  if (!h) return SSSP_ERR_INVALID_ARGUMENT;
  if (n) *n = h->n;
  if (m) *m = h->m;
  if (wtype) *wtype = h->wtype;
  return SSSP_OK;
}

void sssp_destroy(sssp_handle* h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  free_handle(h);
}

}  // extern "C"
