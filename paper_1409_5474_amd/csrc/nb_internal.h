// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nbody.h"

namespace nb {

constexpr int kWG = 256;    // threads per workgroup of the force kernels unless a launch names another
// Threads per workgroup of the batched scalar j-path: its i-block, WG * K
// rows of one system, is half the single-system one, so systems of a few
// hundred rows leave fewer lanes idle in their last i-block
constexpr int kBatchSjWG = 128;
constexpr int kTile = 256;  // j-particles staged in LDS per tile
constexpr int kWorkQueueWords = 16;  // words of a context's work queue (9 used)
constexpr int kMaxSubRegimes = 16;   // active-count regimes one device-count launch can serve
constexpr int kErrorWord = kWorkQueueWords - 1;  // word of that buffer holding the device error bits
constexpr unsigned int kErrActiveRange = 1u;     // an active_idx entry outside its valid range was skipped
constexpr unsigned int kErrTreeStack = 2u;       // a tree walk's stack reached its bound (its group unwritten)

// The range test of every kernel that reads an i-set entry: r must lie in
// [lo, hi).  Host and device share it, so a host test exercises this code.
__host__ __device__ inline bool row_in_range(int64_t r, int64_t lo, int64_t hi) { return r >= lo && r < hi; }

// One launch configuration of the force kernel family.
struct Launch {
  int K = 1;      // i-particles per lane
  int L = 1;      // lanes per i-particle
  int S = 1;      // j-subsets (0: choose by the saturation rule)
  int items = 0;  // work-item target of the saturation rule (0: 4 per CU)
  int fam = 0;    // > 0: run in the LDS kernel family `fam`, which holds this
                  // shape and, in device-count mode, every shape of the call
  int T = kTile;  // j-particles per LDS tile (L >= 1), also the j-chunk quantum
  int WG = kWG;   // threads per workgroup
};

// The LDS tile length and workgroup size every kernel family, the masked
// (eps2 = 0) kernels and the hybrid path are built for.
inline bool default_tile(const Launch& c) { return c.T == kTile && c.WG == kWG; }
// eps2 == 0 runs the masked kernels: one i-particle per lane, default tile.
inline Launch masked(Launch c) {
  c.K = 1;
  c.T = kTile;
  c.WG = kWG;
  return c;
}

// LDS kernel families: one kernel holding the bodies of several (K, L)
// shapes, so that device-count regimes of different shapes share one launch
// (each launch costs a few microseconds in every block step).
//   family 1: K = 1, L in {1, 4, 16, 64, 256}
//   family 2: family 1 and K = 2, L in {1, 4, 16}
//   family 4: family 1 and K = 4, L = 4
// Returns the smallest family holding the shape, 0 for none.
inline int family_of(int K, int L) {
  if (K == 1 && (L == 1 || L == 4 || L == 16 || L == 64 || L == 256)) return 1;
  if (K == 2 && (L == 1 || L == 4 || L == 16)) return 2;
  if (K == 4 && L == 4) return 4;
  return 0;
}
// The smallest family holding both families' shapes (0: none).
inline int family_cover(int a, int b) {
  if (a == 0 || b == 0) return 0;
  if (a == b || b == 1) return a;
  if (a == 1) return b;
  return 0;  // families 2 and 4 hold different K
}
__host__ __device__ constexpr int shape_code(int K, int L) { return (K << 16) | L; }

// i-particles per workgroup of a launch shape (L = 0: the scalar j-path,
// one i-slot per lane like L = 1).
inline int ib_of(const Launch& c) { return (c.WG / (c.L > 0 ? c.L : 1)) * c.K; }

// Lanes that share one output of a j-split sum over S partial blocks: the
// fewest (a power of two, at most a wavefront) with no lane adding more than
// four blocks.  A small active set gets many blocks, and one lane reading
// them all in turn is bound by their load latency.
__host__ __device__ constexpr int chunk_lanes(int S) {
  int g = 1;
  while (g < 64 && 4 * g < S) g <<= 1;
  return g;
}

// The sum of one output over its S blocks p[0], p[stride], ...: `lane` of g
// (g = chunk_lanes(S), the g lanes consecutive and g-aligned in the
// wavefront, all of them calling) adds blocks lane, lane + g, ... in
// ascending order, then a fixed butterfly folds the g sums.  The value lane 0
// returns depends on S alone, not on the launch.
__device__ __forceinline__ double sum_blocks(const double* __restrict__ p, int64_t stride, int S, int lane, int g) {
  double s = 0.0;
  for (int ch = lane; ch < S; ch += g) s += p[(int64_t)ch * stride];
  for (int m = g >> 1; m > 0; m >>= 1) s += __shfl_xor(s, m);
  return s;
}

struct TuneEntry {
  int prec;
  int64_t n_min, act_min, act_max;
  Launch cfg;
};

// Tuned shape of the batched force kernel.  kind 1: nbody_forces_batch,
// keyed by the mean active rows per system; kind 2: the batched block step,
// keyed by the mean system size (the step's count is known only on the
// device).
struct BatchTuneEntry {
  int prec, kind;
  int64_t key_min, key_max;
  Launch cfg;
};

// Arguments of one force launch.  j rows [0, n) of pos/vel/mass; i rows
// active[0, n_active).  When n_active_dev is set the count is read on the
// device and the j-split is chosen there.
struct ForceArgs {
  const double* pos;
  const double* vel;
  const double* mass;
  int64_t n;
  const int32_t* active;
  int64_t n_active;             // host count (or the maximum, with n_active_dev)
  const int32_t* n_active_dev;  // optional device count
  double eps2;
  int S;                        // j-subsets (host-chosen); ignored with n_active_dev
  int target_items;             // device-chosen S aims at this many work items
  double* acc;
  double* jerk;
  double* pot;
  double* part;                 // [S][7][n_active] partial sums when S > 1
  int* s_dev;                   // device count: the working regime's S, for the shared reduce
  int64_t act_lo;               // device-count mode: work only when count >= act_lo and
  int last;                     // count <= n_active (or any larger count when `last`)
  // Device-count mode, one launch serving several adjacent regimes of one
  // shape: regime r starts at count sub_lo[r] and aims at sub_items[r] work
  // items, so the count picks the same S as a host-count launch would
  // (n_sub == 0: target_items for every count).
  int n_sub;
  int64_t sub_lo[kMaxSubRegimes];
  int sub_items[kMaxSubRegimes];
  // Family launches: the shape (shape_code) of the call, and in device-count
  // mode that of regime r (the regimes of one launch may differ in shape).
  int shape;
  int sub_shape[kMaxSubRegimes];
  void* rec;                    // scalar j-path: mirror of n j-records (context-owned)
  // Work queue of the persistent grid (per-XCD item counters, then the count
  // of finished workgroups): zero before a launch, and the launch's last
  // workgroup sets it back to zero (context-owned, kWorkQueueWords words).
  unsigned int* wq;
  // Receiving particles given apart from the j-set: `active` then indexes
  // ipos/ivel (null: the j arrays) and, with no_self set, no self pair is
  // removed from the potential (the i-set is not part of the j-set).
  const double* ipos;
  const double* ivel;
  int no_self;
  // Valid i-set entries lie in [row_lo, row_hi): others are skipped (no
  // output row is written for them) and set kErrActiveRange in *err.
  int64_t row_lo, row_hi;
  unsigned int* err;
};

// Arguments of the sixth-order force kernel (forces6.hip): acceleration,
// jerk, snap and potential of the active rows, every particle moving with
// its own position, velocity and (predicted) acceleration accj.
struct Force6Args {
  const double* pos;
  const double* vel;
  const double* accj;
  const double* mass;
  int64_t n;
  const int32_t* active;
  int64_t n_active;             // host count (or the maximum, with n_active_dev)
  const int32_t* n_active_dev;  // optional device count
  double eps2;
  int S;                        // j-chunks (host count only)
  int target_items;             // device count: chunks chosen for this many items
  double* acc;
  double* jerk;
  double* snap;
  double* pot;
  double* part;                 // [S][10][n_active] partial sums when S > 1
  unsigned int* err;            // i-set entries outside [0, n) are skipped and flagged here
};

// Batched work list item: one (system, i-block, j-chunk) triple.
struct BatchItem {
  int32_t sys;      // system index
  int32_t iblk;     // i-block inside the system's active list
  int32_t chunk;    // j-chunk inside the system
  int32_t nchunk;   // number of chunks of this system
};

struct BatchSys {
  int64_t j0, j1;     // j rows of the system
  int64_t a0, a1;     // rows of the active list / outputs
  double eps2;
  int64_t part_off;   // offset (in rows of 7 doubles) of its partials
};

// Kernel launchers (forces.hip).  Return hipSuccess or the launch error.
hipError_t launch_forces(int prec, const Launch& cfg, bool mask, const ForceArgs& a, hipStream_t st,
                         int grid_override, int max_grid);
int resident_wgs(int prec, const Launch& cfg, bool mask);
// The paper's atomic alternative to the two-kernel j-split sum (LDS kernel
// families 1 and 2, eps2 > 0): outputs seeded, then every work item adds
// its partial sums with device-scope atomics.
bool atomic_split_supported(const Launch& c);
hipError_t launch_forces_atomic(int prec, const Launch& cfg, const ForceArgs& a, hipStream_t st, int max_grid);
size_t mirror_bytes(int prec, int64_t n);  // j-record mirror of the scalar j-path
hipError_t launch_reduce_ib(int prec, const ForceArgs& a, int S, int IB, hipStream_t st);
int host_choose_S(int64_t n_act, int IB, int target_items, int64_t n, int tile);
bool launch_supported(const Launch& cfg);
int items_for(const Launch& cfg, int64_t n_active, int S);
hipError_t launch_batch(int prec, const Launch& cfg, const BatchItem* items, int n_items, const int* n_items_dev,
                        const BatchSys* sys, const double* pos, const double* vel, const double* mass,
                        const int32_t* active, double* acc, double* jerk, double* pot, double* part,
                        int64_t part_rows, bool any_mask, int max_grid, unsigned int* err, void* rec,
                        int64_t n_total, hipStream_t st);
// whether the batched force kernel exists in this shape (L = 0: scalar j-path)
bool batch_supported(const Launch& c);
// Workgroups per CU the batched force kernel of this shape holds at once.
int batch_resident_wgs(int prec, const Launch& cfg, bool mask);
hipError_t launch_batch_plan(const int64_t* off, const double* eps2, int C, const int32_t* active,
                             const int64_t* n_act_dev, int IB, int target, BatchSys* sys, int32_t* nchunk,
                             BatchItem* items, int max_items, int* n_items_dev, int64_t part_cap_rows,
                             hipStream_t st);
hipError_t launch_batch_reduce(int prec, const BatchSys* sys, int n_sys, const int32_t* chunks_per_sys,
                               const double* mass, const int32_t* active, int64_t n_act_total,
                               double* acc, double* jerk, double* pot, const double* part,
                               hipStream_t st);

// Hermite / schedule / energy launchers (hermite.hip).
hipError_t launch_predict(const double* pos, const double* vel, const double* acc, const double* jerk,
                          const int64_t* t_tick, int64_t t_next, const int64_t* t_next_dev, double dt_min,
                          int64_t n, double* pos_p, double* vel_p, hipStream_t st);
hipError_t launch_correct(const int32_t* active, int64_t n_active, const int64_t* n_active_dev, int64_t n_rows,
                          unsigned int* err, const double* pos_p, const double* vel_p, const double* acc1,
                          const double* jerk1, double* pos, double* vel, double* acc, double* jerk,
                          int64_t* t_tick, int32_t* level, double eta, double dt_max, int max_level,
                          int64_t* clamp_dev, hipStream_t st);
hipError_t launch_correct_step(const int32_t* active, int64_t n_max, const int64_t* n_active_dev, int64_t n_rows,
                               unsigned int* err, const double* pos_p, const double* vel_p, const double* acc1,
                               const double* jerk1, double* pos, double* vel, double* acc, double* jerk,
                               int64_t* t_tick, int32_t* level, double eta, double dt_max, int max_level,
                               int64_t* clamp_dev, int64_t* step_dev, hipStream_t st);
hipError_t launch_startup(const double* acc, const double* jerk, int64_t n, double eta, double dt_max,
                          int max_level, int32_t* level, hipStream_t st);
// The Hermite state a block step corrects after its force pass (the fused
// reduce-and-correct kernel): predicted and current positions, velocities,
// accelerations, jerks, ticks and levels of all particles, the step
// parameters, and the device counters of clamped levels and of steps.
struct StepArgs {
  const double* pos_p;
  const double* vel_p;
  double* pos;
  double* vel;
  double* acc;
  double* jerk;
  int64_t* t_tick;
  int32_t* level;
  double eta, dt_max;
  int max_level;
  unsigned long long* clamp_dev;
  unsigned long long* step_dev;
};
hipError_t launch_reduce_correct(int prec, const ForceArgs& a, const StepArgs& s, hipStream_t st);
// the same for a batched block step (rows of every system, device count)
hipError_t launch_batch_reduce_correct(int prec, const BatchSys* sys, const int32_t* chunks_per_sys, int C,
                                       const int64_t* n_act_dev, int64_t n_max, const double* mass,
                                       const int32_t* active, double* acc1, double* jerk1, double* pot1,
                                       const double* part, const StepArgs& s, unsigned int* err, hipStream_t st);

// The predictor folded into the scheduler's last pass (all pointers null:
// no prediction).  Predicts every particle to the scheduled t_next.
struct PredictArgs {
  const double* pos;
  const double* vel;
  const double* acc;
  const double* jerk;
  double dt_min;
  double* pos_p;
  double* vel_p;
};
hipError_t launch_schedule(const int64_t* t_tick, const int32_t* level, int64_t n, int max_level,
                           int32_t* active, int64_t* sched, int64_t* block_min, int32_t* block_cnt,
                           int32_t* n_active32, int64_t t_stop, const int64_t* t_stop_dev, hipStream_t st,
                           const PredictArgs* pred = nullptr);
int schedule_blocks(int64_t n);
hipError_t launch_energy(const double* pos, const double* vel, const double* mass, const double* pot,
                         int64_t n, double* part, double* out, hipStream_t st);
int energy_blocks(int64_t n);

// Tree code (tree.hip).
struct TreeCell {
  int32_t begin, end;      // range of the cell's particles along the curve
  int32_t child0, nchild;  // children are contiguous; nchild == 0 for a leaf
  int32_t level, pad;
  double corner[3];        // cube corner and side
  double side;
  double M;                // mass, centre of mass, traceless quadrupole
  double X[3];
  double Q[6];             // xx, yy, zz, xy, xz, yz
};
struct TreeStats {
  int64_t cells, groups, accepted, opened_leaves;
  int depth;
};
// Device buffers of the tree code, grown on demand and kept between calls.
struct TreeScratch {
  std::vector<std::pair<void*, size_t>> slots;
  void* host = nullptr;    // pinned, for the per-level counts
};
// The whole evaluation is enqueued without host reads; with `stats` set it
// then synchronises and reads the counts (and reports a stack overflow as
// hipErrorInvalidValue).  `capturing`: no buffer may grow (a call outside the
// capture sizes them); a stack overflow is then flagged in *err only.
hipError_t tree_forces_run(TreeScratch& s, hipStream_t st, const double* pos, const double* mass, int32_t n,
                           double eps2, double theta, int n_crit, double g_frac, bool mixed, double* acc,
                           double* pot, TreeStats* stats, bool capturing, unsigned int* err, const char** msg);
// The Peano-Hilbert keys of the positions in curve order and the input row
// of each (the tree code's first stage).
hipError_t tree_sorted_keys(TreeScratch& s, hipStream_t st, const double* pos, int32_t n, uint64_t* keys_out,
                            int32_t* idx_out, const char** msg);
void tree_scratch_free(TreeScratch& s);

// Sixth-order force kernel (forces6.hip).
int forces6_resident_wgs(bool mask);
int forces6_split(int64_t n_act, int target_items, int64_t n);
int64_t forces6_workspace_rows(int64_t n_max, int target_items, int64_t n);
hipError_t launch_forces6(const Force6Args& a, bool mask, int grid, hipStream_t st);

// Sixth-order Hermite passes (hermite6.hip).
hipError_t launch_predict6(const double* pos, const double* vel, const double* acc, const double* jerk,
                           const double* snap, const double* crackle, const int64_t* t_tick, int64_t t_next,
                           const int64_t* t_next_dev, double dt_min, int64_t n, double* pos_p, double* vel_p,
                           double* acc_p, hipStream_t st);
hipError_t launch_correct6(const int32_t* active, int64_t n_max, const int64_t* n_active_dev, int64_t n_rows,
                           unsigned int* err, const double* acc1, const double* jerk1, const double* snap1,
                           double* pos, double* vel, double* acc, double* jerk, double* snap, double* crackle,
                           int64_t* t_tick, int32_t* level, double eta, double dt_max, int max_level,
                           int64_t* clamp_dev, int64_t* step_dev, hipStream_t st);
hipError_t launch_startup6(const double* acc, const double* jerk, const double* snap, int64_t n, double eta_s,
                           double dt_max, int max_level, int32_t* level, hipStream_t st);

// Kick / kick-drift passes of the Hamiltonian split (bridge.hip).
hipError_t launch_kick(double* vel, const double* acc, double h, int64_t n, hipStream_t st);
hipError_t launch_kick_drift(double* pos, double* vel, const double* acc, double h_kick, double h_drift, int64_t n,
                             hipStream_t st);

}  // namespace nb

// The context behind the opaque handle of the C ABI.
struct nb_ctx {
  int device = 0;
  int prec = NB_PREC_FP64;
  int num_cus = 256;
  hipStream_t stream = nullptr;
  std::string err;
  nb::Launch forced;            // K == 0: automatic
  bool have_forced = false;
  bool split_atomic = false;      // nb_set_split_sum: host-count j-split sums by atomics
  std::vector<nb::TuneEntry> table;
  std::vector<nb::BatchTuneEntry> batch_table;
  // device workspace (grown on demand)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* mirror = nullptr;       // j-records of the scalar j-path
  size_t mirror_bytes = 0;
  int* s_dev = nullptr;         // S chosen on the device by the last device-count launch
  unsigned int* wq = nullptr;   // work queue of the force grids (zero between launches)
  int64_t* sched_tmp = nullptr; // block minima for the scheduler
  int32_t* sched_cnt = nullptr;
  int32_t* nact32 = nullptr;    // int32 copy of the scheduled active count
  size_t sched_cap = 0;
  double* energy_part = nullptr;
  size_t energy_cap = 0;
  void* batch_buf = nullptr;    // device copy of the batch work list
  size_t batch_cap = 0;
  void* batch_host = nullptr;   // pinned staging buffer of the work list
  size_t batch_host_cap = 0;
  hipEvent_t batch_ev = nullptr;  // marks the end of the last staging copy
  // device-planned batch block steps: system table and work list
  std::vector<int64_t> bp_off;    // host copy of the uploaded offsets
  std::vector<double> bp_eps2;    // host copy of the uploaded softenings
  nb::TreeScratch tree;           // buffers of the tree code
  const int64_t* stop_dev = nullptr;  // block steps read their stop tick here when set
  void* bp_buf = nullptr;         // offsets, eps2, sys, nchunk, items, n_items
  size_t bp_cap = 0;
  int bp_max_items = 0;
  int log_level = 0;              // NB_LOG at nb_create: 0 silent, 1 errors, 2 also launch choices
  // phase timing of eager block steps (nb_set_phase_timing): events at the
  // start, after the schedule (and plan), after the forces, after the corrector
  bool phase_on = false;
  bool phase_valid = false;       // the last block step recorded all four
  hipEvent_t phase_ev[4] = {};
};
