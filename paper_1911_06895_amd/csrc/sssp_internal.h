// Internal declarations shared by the kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sssp {

constexpr int kWG = 1024;              // larger solver workgroup (on request; the adjoint's): 16 wave64s, one per CU
constexpr int kWGGroups = 512;         // default solver workgroup: 8 wave64s, two per CU
constexpr int kAuxWG = 256;            // workgroup of the create-time kernels
constexpr uint32_t kChunk = 512;       // most list entries a workgroup expands at a time (LDS tile bound)
constexpr uint32_t kMinChunk = 32;     // fewest list entries per claimed chunk
constexpr uint32_t kILP = 2;           // edges per lane per round (2 measured faster than 3, 4 and 8)
constexpr uint32_t kPieceMin = kWGGroups * kILP;  // edges of the smaller hub piece (one round of a workgroup)
constexpr uint32_t kHub = 1024;        // default: a vertex with at least this many edges in a phase goes to the hub step
constexpr uint32_t kHubMin = 256;      // smallest hub threshold a tuning may set (sizes the hub queues)
constexpr uint32_t kBarGroups = 8;     // arrival sub-counters of the grid barrier
constexpr uint32_t kRingMax = 64;      // near-bucket ring capacity
constexpr uint32_t kDegClasses = 65536;  // in-degree classes of the relabelling (the last one open-ended)
constexpr uint32_t kMaxGroups = 256;   // concurrent sources of one launch (workgroup groups)
constexpr uint32_t kEpochLimit = 1u << 30;  // de-duplication tags are reset before they pass this
constexpr uint32_t kNone = 0xFFFFFFFFu;

// Tentative distances are kept as unsigned bit patterns: uint32 values for
// integer weights, and for fp32 (fp64) weights the IEEE bits of non-negative
// floats, which order exactly like the floats themselves (+0.0 = 0, +inf =
// 0x7F800000, resp. 0x7FF0000000000000).
constexpr uint32_t kInfU32 = 0xFFFFFFFFu;
constexpr uint32_t kInfF32 = 0x7F800000u;
constexpr uint64_t kInfF64 = 0x7FF0000000000000ull;

enum WeightType : int { kWU32 = 0, kWF32 = 1, kWF64 = 2 };

// The light/heavy threshold delta in the weight type's own terms.
struct Threshold {
  int wtype;
  uint32_t delta_u;  // integer weights
  float delta_f;     // fp32 weights
  double delta_d;    // fp64 weights
};

// Weight e of a caller array as bits (zero-extended for 32-bit types).
__device__ inline uint64_t weight_bits(const void* w, int wtype, int64_t e) {
  return wtype == kWF64 ? static_cast<const uint64_t*>(w)[e] : static_cast<uint64_t>(static_cast<const uint32_t*>(w)[e]);
}

// A usable weight: integers >= 1; floats finite and > 0 (no sign bit, not
// +0.0, exponent not all ones).
__device__ inline bool weight_ok(uint64_t wb, int wtype) {
  if (wtype == kWU32) return wb != 0;
  if (wtype == kWF32) return !((wb & 0x80000000u) || wb == 0 || (wb & 0x7F800000u) == 0x7F800000u);
  return !((wb >> 63) || wb == 0 || ((wb >> 52) & 0x7FFu) == 0x7FFu);
}

__device__ inline double weight_value(uint64_t wb, int wtype) {
  if (wtype == kWU32) return static_cast<double>(wb);
  if (wtype == kWF32) return static_cast<double>(__uint_as_float(static_cast<uint32_t>(wb)));
  return __longlong_as_double(static_cast<long long>(wb));
}

// light: w <= delta (A_L = A o (0 < A <= delta), Sec. IV-A)
__device__ inline bool is_light(uint64_t wb, const Threshold& th) {
  if (th.wtype == kWU32) return wb <= th.delta_u;
  if (th.wtype == kWF32) return __uint_as_float(static_cast<uint32_t>(wb)) <= th.delta_f;
  return __longlong_as_double(static_cast<long long>(wb)) <= th.delta_d;
}

enum Action : uint32_t {
  kActLight = 1,  // light phase over the current frontier
  kActHeavy = 2,  // heavy phase over S
  kActFar = 3,    // move far-future vertices into the ring
  kActDone = 4,
  kActOverflowCheck = 5,
  kActHub = 6,    // pieces of high-degree vertices left over by the previous phase
};

enum InKind : uint32_t { kInF0 = 0, kInF1 = 1, kInBin = 2 };

// Device control block of the persistent solver. The barrier words and the
// epoch counters persist across launches; the schedule fields are set by the
// barrier leader (the last workgroup to arrive) before it releases the others,
// so every workgroup reads the same schedule.
struct Ctl {
  // grid barrier: arrival sub-counters on separate 128-byte lines, then the top counter
  uint32_t bar_sub[kBarGroups][32];
  // Fields that different workgroups update or poll at the same time sit on
  // separate 128-byte lines, so atomics on one do not queue behind traffic to another.
  alignas(128) uint32_t bar_arrive;
  alignas(128) uint32_t bar_gen;  // polled by the waiting workgroups
  uint32_t abort;
  uint32_t heartbeat;     // bumped by the leader at each step it runs alone inside a barrier
  uint32_t source_index;  // source (row) the group is solving, kNone when the batch is done
  alignas(128) uint32_t chunk_next;  // dynamic chunk counter of the current step
  alignas(128) uint32_t hub_count;   // hub pieces queued by the current phase
  alignas(128) uint32_t hub_next;    // dynamic claim counter of the pieces processed by the current step
  // schedule of the pieces processed by the current step
  alignas(128) uint32_t hub_parent;  // action of the phase that queued them
  uint32_t hub_backlog;  // pieces to process (a hub step, or a light phase finishing the previous one's)
  uint32_t hub_in;       // queue buffer holding them; a phase appends to the other one
  uint32_t redo;         // the current round repeats its bucket (fp32 heavy requests fell back into it)
  // schedule
  alignas(128) uint32_t action;
  uint32_t bucket;       // current bucket i
  uint32_t in_kind;      // InKind of the current input list
  uint32_t in_count;     // entries in the current input list
  uint32_t out_buf;      // frontier buffer receiving re-inserted vertices (0/1)
  uint32_t far_base;     // ring base used by a far redistribution
  uint32_t step;         // frontier de-duplication tag (monotone across solves)
  uint32_t round;        // S de-duplication tag (monotone across solves)
  uint32_t far_epoch;    // far-list de-duplication tag (monotone across solves)
  uint32_t far_cur;      // which far list is current (0/1)
  // bounds [lo, hi) of the current bucket (integer weights)
  uint64_t lo_u, hi_u;
  // counters
  alignas(128) uint32_t far_min;  // lower bound on the bucket of any far vertex
  uint32_t far_min_next;
  alignas(128) uint32_t fcount[2];
  alignas(128) uint32_t scount;
  alignas(128) uint32_t farcount[2];
  alignas(128) uint32_t ovf_seen;  // some candidate did not fit the distance type
  uint32_t ovf_real;     // a reachable vertex has an unrepresentable distance (adjoint: dist is not a
                         // shortest-path vector)
  uint32_t trace_len;    // step records written (may exceed trace_cap)
  unsigned long long* trace;  // optional step trace: 4 words per record
  unsigned long long tr_edges, tr_impr;  // edges scanned and improvements of the running step (traced runs)
  uint32_t trace_cap;
  uint32_t next_source;  // batch-wide source counter (used in the first group's block only)
  uint32_t bad_source;   // a source index outside [0, n) was given
  uint32_t hub_full;     // a hub queue ran out of room (the schedule was aborted)
  unsigned long long wait_ticks;  // a barrier wait without progress longer than this aborts the schedule
  alignas(128) uint32_t bincount[kRingMax][32];  // ring-slot sizes, one per 128-byte line ([slot][0])
  // statistics (summed over sources)
  alignas(128) unsigned long long sources, buckets, light_phases, heavy_phases, far_phases;
  unsigned long long light_edges, heavy_edges, improvements, attempts, barriers;
  unsigned long long adj_released;  // adjoint: vertices released (equals the reached count)
};

struct Params {
  uint32_t n;
  uint32_t ring;        // ring size, power of two
  uint32_t ring_mask;
  uint32_t wtype;       // 0 = u32, 1 = f32
  uint32_t delta_u;     // u32 delta
  double delta_d;       // f32: (double)(float)delta; f64: delta
  double inv_delta_d;   // 1 / delta_d (an estimate; bucket indices are corrected exactly)
  const uint32_t* vid;    // [n] solver id of each caller vertex (decreasing in-degree order)
  uint32_t zero_from;     // solver ids from here on have no in-edges (reachable only as a seed)
  void* tbuf[2];          // [n] 64-bit tentative-distance words in solver ids (alternating between sources)
  void* texp;             // fp64: [n] distance of each vertex at its last light expansion in the current row
  const uint4* rows;      // [n] row u of the split copy: (start, end of light edges, end, 0)
  const uint64_t* edges;  // [m] (destination | weight bits << 32); fp64: destination only
  const uint64_t* w64;    // [m] fp64 weight bits at the same positions (fp64 handles)
  uint32_t* qstamp;       // [n] frontier tag of the last push
  uint32_t* sstamp;       // [n] round tag of the last S insertion
  uint32_t* bstamp;       // [n] a bucket the vertex was filed under in the ring (this solve; kNone: none)
  uint32_t* fstamp;       // [n] far epoch of the last far insertion
  uint32_t* ovf_at;       // [n] a candidate for this vertex did not fit
  uint32_t* front[2];     // [n] frontier buffers
  uint32_t* slist;        // [n] S
  uint32_t* bins;         // [ring][n]
  uint32_t* far[2];       // [n] far lists
  uint64_t* hub;          // [2][hub_cap] pieces (vertex | piece index << 32), two alternating queues
  uint32_t hub_cap;
  uint32_t inline_edges;  // steps with at most this many edges run on the leader workgroup alone
  uint32_t hub_edges;     // a vertex with at least this many edges in a phase is cut into hub pieces
  uint32_t chunk_entries; // list entries per claimed chunk at most (power of two <= kChunk; 0: by group size)
  uint32_t inline_entries;  // list entries of a step the leader runs alone at most (<= kChunk; 0: the chunk cap)
  uint32_t groups;        // workgroup groups of the launch, each solving its own sources
  uint32_t no_heavy;      // every weight is <= delta: A_H is empty, no S and no heavy phases
  Ctl* ctl;               // this group's control block
  uint32_t* next_source;  // shared by every group: next source row to claim
};

// Adjoint working set (solver ids unless noted).
struct AdjParams {
  uint32_t n;
  uint64_t m;
  const uint32_t* vid;        // [n] caller -> solver id
  const uint32_t* inv;        // [n] solver -> caller id
  const uint4* rows;
  const uint64_t* edges;
  const uint32_t* perm;       // packed position -> caller edge index
  uint32_t* d;                // [n] distances
  unsigned long long* parent; // [n] (caller edge index << 32 | parent solver id), all ones = none
  uint32_t* cnt;              // [n] children still to report
  uint32_t* lvl;              // [n] round in which a vertex got its parent (kNone: unresolved)
  double* g;                  // [n] accumulated coefficients
  uint32_t* front[2];         // [n] level lists
  double* grad64;             // [m] dL/dw in caller edge order (shared by every group)
  Ctl* ctl;                   // this group's control block
  uint32_t* next_source;      // shared by every group: next source row to claim
};

// launchers (sssp_kernels.hip, sssp_adjoint.hip, sssp_build.hip)
hipError_t adjoint_occupancy(int* blocks_per_cu);
// `params`: device array of one AdjParams per group; grad64 is zeroed first and
// converted into grad_w (fp32) after the launch.
hipError_t launch_adjoint(const AdjParams* params, uint32_t groups, const int32_t* sources, int k, const uint32_t* dist,
                          const float* grad_dist, float* grad_w, uint64_t m, double* grad64, int grid, hipStream_t s);
hipError_t launch_count_reached(const uint32_t* dist, uint32_t n, int k, int wtype, unsigned long long* out,
                                hipStream_t s);
hipError_t launch_resplit(uint32_t n, const uint4* rows_in, const uint64_t* edges_in, const uint32_t* perm_in,
                          const void* w, const Threshold& th, uint4* rows_out, uint64_t* w64_out,
                          uint64_t* edges_out, uint32_t* perm_out, hipStream_t s);
hipError_t launch_inverse(const uint32_t* vid, int64_t n, uint32_t* inv, hipStream_t s);
hipError_t launch_validate_weights(const void* w, int wtype, int64_t m, uint32_t* status, unsigned long long* wmax_bits,
                                   double* wsum, hipStream_t s);
hipError_t launch_validate(const int64_t* row_ptr, const int32_t* col, const void* w, int wtype, int64_t n,
                           int64_t m, uint32_t* status, unsigned long long* wmax_bits, double* wsum, hipStream_t s);
size_t build_scratch_words(int64_t n);
// After launch_relabel_and_split, this word of its scratch holds the number of vertices without
// in-edges (the in-degree histogram's first class; their solver ids come last).
inline size_t relabel_no_in_edges_word(int64_t n) { return static_cast<size_t>(n); }
hipError_t launch_relabel_and_split(const int64_t* row_ptr, const int32_t* col, const void* w, const Threshold& th,
                                    int64_t n, int64_t m, uint32_t* scratch,
                                    uint32_t* new_id, uint32_t* off, uint32_t* split, uint64_t* edges,
                                    uint64_t* w64, uint32_t* perm, hipStream_t s);
hipError_t solver_occupancy(int wtype, int wg, bool chain, int* blocks_per_cu);
hipError_t launch_pack_rows(const uint32_t* off, const uint32_t* split, int64_t n, uint4* rows, hipStream_t s);
hipError_t launch_ctl_reset(Ctl* c, uint32_t groups, int reset_epochs, unsigned long long* trace, uint32_t trace_cap,
                            unsigned long long wait_ticks, hipStream_t s);
hipError_t launch_fill(uint32_t* p, size_t count, uint32_t value, hipStream_t s);
// `params` is a device array of one Params per group; grid must be a multiple of
// groups; wg (kWG or kWGGroups) is the workgroup size; chain: the kernel whose
// leader chains its light steps. multi = 0: row r of dist holds the distances
// from sources[r]; multi = 1: one row, the distances from the nearest of the k
// sources.
hipError_t launch_solver(const Params* params, uint32_t groups, uint32_t wtype, const int32_t* sources, int k,
                         int multi, void* dist, int grid, int wg, bool chain, hipStream_t s);

// validation status bits
enum : uint32_t {
  kBadRowPtr = 1u,
  kBadCol = 2u,
  kBadWeight = 4u,
};

}  // namespace sssp
