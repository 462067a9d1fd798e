// C ABI of the library: argument checking, launch-configuration choice,
// workspace management and the composite block step.  See include/nbody.h.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>

#include "nb_internal.h"

using nb::Launch;

namespace {

constexpr const char* kVersion = "nbody-mi355x 0.1 (gfx950)";

// NB_LOG (read by nb_create): 1 prints every error a call returns, 2 also
// each host-side launch choice; lines go to stderr, prefixed "nbody:".
int log_level_from_env() {
  const char* v = std::getenv("NB_LOG");
  if (!v || !*v) return 0;
  const int l = std::atoi(v);
  return l < 0 ? 0 : l;
}

int fail(nb_ctx* c, int code, const char* fmt, const char* detail = nullptr) {
  if (c) {
    char buf[512];
    std::snprintf(buf, sizeof buf, fmt, detail ? detail : "");
    c->err = buf;
    if (c->log_level >= 1) std::fprintf(stderr, "nbody: error %d: %s\n", code, buf);
  }
  return code;
}

int hip_fail(nb_ctx* c, hipError_t e, const char* where) {
  char buf[512];
  std::snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
  if (c) {
    c->err = buf;
    if (c->log_level >= 1) std::fprintf(stderr, "nbody: error %d: %s\n", NB_EDEVICE, buf);
  }
  return NB_EDEVICE;
}

void log_launch(const nb_ctx* c, const char* what, const Launch& cfg, int64_t N, int64_t n_active) {
  if (c->log_level < 2) return;
  std::fprintf(stderr, "nbody: %s N=%lld n_active=%lld K=%d L=%d S=%d T=%d WG=%d items=%d\n", what, (long long)N,
               (long long)n_active, cfg.K, cfg.L, cfg.S, cfg.T, cfg.WG, cfg.items);
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

// Phase event k of an eager block step (0: start, 1: after the schedule and
// plan, 2: after the forces, 3: after the corrector).  Steps inside a graph
// capture record nothing and leave the last eager step's times in place.
void phase_mark(nb_ctx* c, int k) {
  if (!c->phase_on) return;
  if (k == 0) {
    if (capturing(c->stream)) return;
    c->phase_valid = false;
  } else if (!c->phase_ev[0] || capturing(c->stream)) {
    return;
  }
  if (hipEventRecord(c->phase_ev[k], c->stream) != hipSuccess) {
    (void)hipGetLastError();
    c->phase_valid = false;
    return;
  }
  if (k == 3) c->phase_valid = true;
}

// Optional cap on the j-split workspace and on the j-record mirror
// (environment NB_MAX_WORKSPACE_BYTES): a request above it fails with
// NB_ENOMEM instead of allocating.
size_t workspace_cap() {
  const char* v = std::getenv("NB_MAX_WORKSPACE_BYTES");
  if (!v || !*v) return SIZE_MAX;
  char* end = nullptr;
  const unsigned long long x = std::strtoull(v, &end, 10);
  return (end && *end == '\0') ? (size_t)x : SIZE_MAX;
}

// Grow the context workspace to at least `bytes` (never inside a capture).
int ensure_ws(nb_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return NB_OK;
  if (bytes > workspace_cap())
    return fail(c, NB_ENOMEM, "j-split workspace request exceeds NB_MAX_WORKSPACE_BYTES%s");
  if (capturing(c->stream))
    return fail(c, NB_ENOMEM, "workspace must grow but the stream is being captured; run the call once before capture%s");
  if (c->ws) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  // grow with some headroom, but never past the cap
  size_t b = bytes + bytes / 4;
  if (b > workspace_cap()) b = workspace_cap();
  if (hipMalloc(&c->ws, b) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, NB_ENOMEM, "hipMalloc of the j-split workspace failed%s");
  }
  c->ws_bytes = b;
  return NB_OK;
}

// The j-record mirror of the scalar j-path (L = 0), grown on demand.
int ensure_mirror(nb_ctx* c, int64_t n) {
  const size_t bytes = nb::mirror_bytes(c->prec, n);
  if (bytes <= c->mirror_bytes) return NB_OK;
  if (bytes > workspace_cap())
    return fail(c, NB_ENOMEM, "j-record mirror exceeds NB_MAX_WORKSPACE_BYTES%s");
  if (capturing(c->stream)) return fail(c, NB_ENOMEM, "j-record mirror must grow during capture%s");
  (void)hipStreamSynchronize(c->stream);
  if (c->mirror) (void)hipFree(c->mirror);
  c->mirror = nullptr;
  c->mirror_bytes = 0;
  if (hipMalloc(&c->mirror, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, NB_ENOMEM, "hipMalloc of the j-record mirror failed%s");
  }
  c->mirror_bytes = bytes;
  return NB_OK;
}

int ensure_sched(nb_ctx* c, int64_t n) {
  const int nblk = nb::schedule_blocks(n);
  const size_t need = (size_t)nblk;
  if (need <= c->sched_cap && c->nact32) return NB_OK;
  if (capturing(c->stream)) return fail(c, NB_ENOMEM, "scheduler scratch must grow during capture%s");
  (void)hipStreamSynchronize(c->stream);
  if (c->sched_tmp) (void)hipFree(c->sched_tmp);
  if (c->sched_cnt) (void)hipFree(c->sched_cnt);
  if (c->nact32) (void)hipFree(c->nact32);
  c->sched_tmp = nullptr; c->sched_cnt = nullptr; c->nact32 = nullptr; c->sched_cap = 0;
  if (hipMalloc(&c->sched_tmp, need * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&c->sched_cnt, need * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->nact32, sizeof(int32_t)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, NB_ENOMEM, "hipMalloc of scheduler scratch failed%s");
  }
  c->sched_cap = need;
  return NB_OK;
}

int ensure_energy(nb_ctx* c, int64_t n) {
  const size_t need = (size_t)nb::energy_blocks(n) * 8;
  if (need <= c->energy_cap) return NB_OK;
  if (capturing(c->stream)) return fail(c, NB_ENOMEM, "energy scratch must grow during capture%s");
  (void)hipStreamSynchronize(c->stream);
  if (c->energy_part) (void)hipFree(c->energy_part);
  c->energy_part = nullptr; c->energy_cap = 0;
  if (hipMalloc(&c->energy_part, need * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, NB_ENOMEM, "hipMalloc of energy scratch failed%s");
  }
  c->energy_cap = need;
  return NB_OK;
}

bool valid_prec(int p) { return p == NB_PREC_FP64 || p == NB_PREC_MIXED || p == NB_PREC_MIXED_DS; }

bool valid_K(int K) { return K >= 1 && K <= 4; }  // K = 3 exists for the scalar j-path only
// L = 0 selects the scalar j-path (i-parallel, j-records through the scalar
// cache); L = -1 the hybrid path (positions through the scalar cache,
// velocities and masses through LDS; mixed precision, else as L = 0)
bool valid_L(int L) { return L == 0 || L == -1 || (L >= 1 && L <= 256 && (L & (L - 1)) == 0); }

// Workgroups the whole chip holds at once for this kernel shape.
int resident_grid(const nb_ctx* c, const Launch& cfg, bool mask) {
  return c->num_cus * nb::resident_wgs(c->prec, cfg, mask);
}

// Default work-item target: four items per resident workgroup, so a
// persistent grid of resident workgroups walks equal shares of the work.
int default_items(const nb_ctx* c, const Launch& cfg) { return 4 * resident_grid(c, cfg, false); }

// Built-in choice before any tuning: the i-parallel layout when the active
// set alone fills the chip, more lanes per i-particle as it shrinks.
struct Regime {
  int64_t lo, hi;
  Launch cfg;
};
constexpr int64_t kSmallSystem = 16384;  // untuned systems up to this N: one launch shape
const Regime kDefaultRegimes[5] = {{0, 127, Launch{1, 64, 0, 0}},
                                   {128, 1023, Launch{1, 16, 0, 0}},
                                   {1024, 8191, Launch{1, 4, 0, 0}},
                                   {8192, 65535, Launch{1, 1, 0, 0}},
                                   {65536, INT64_MAX, Launch{2, 1, 0, 0}}};

// The active-count regimes of this context and precision: the tuned table
// entries that apply to N (later entries override earlier ones on their
// range), else the built-in breakpoints.  Regimes tile [0, inf).  A system
// of at most kSmallSystem particles without tuned entries takes one shape
// for every count: its force work is a few microseconds, so in a block step
// the empty launches of other regimes would cost more than the shape loses
// (K = 1, L = 16 stays within 1.3x of the best shape from 1 to N active at
// N = 3899 and 16384); host-count launches use the same rule, so both paths
// split the work identically.
std::vector<Regime> regimes(const nb_ctx* c, int64_t n) {
  bool tuned = false;
  for (const nb::TuneEntry& e : c->table)
    if (e.prec == c->prec && n >= e.n_min) tuned = true;
  if (!tuned && n <= kSmallSystem) return {Regime{0, INT64_MAX, Launch{1, 16, 0, 0}}};
  std::vector<Regime> r(std::begin(kDefaultRegimes), std::end(kDefaultRegimes));
  for (const nb::TuneEntry& e : c->table) {
    if (e.prec != c->prec || n < e.n_min) continue;
    std::vector<Regime> out;
    for (const Regime& g : r) {
      if (g.hi < e.act_min || g.lo > e.act_max) {
        out.push_back(g);
        continue;
      }
      if (g.lo < e.act_min) out.push_back(Regime{g.lo, e.act_min - 1, g.cfg});
      if (g.hi > e.act_max) out.push_back(Regime{e.act_max + 1, g.hi, g.cfg});
    }
    out.push_back(Regime{e.act_min, e.act_max, e.cfg});
    std::sort(out.begin(), out.end(), [](const Regime& a, const Regime& b) { return a.lo < b.lo; });
    r.swap(out);
  }
  return r;
}

// Resolve K, L and the work-item target for an active count; S is then the
// saturation rule unless a forced configuration fixes it.
Launch choose(const nb_ctx* c, int64_t n, int64_t n_act) {
  Launch cfg;
  if (c->have_forced) {
    cfg = c->forced;
  } else {
    for (const Regime& g : regimes(c, n))
      if (n_act >= g.lo && n_act <= g.hi) cfg = g.cfg;
  }
  if (cfg.items <= 0) cfg.items = default_items(c, cfg);
  const int IB = nb::ib_of(cfg);
  const int tile = cfg.L > 0 ? cfg.T : nb::kTile;
  if (cfg.S <= 0) cfg.S = nb::host_choose_S(n_act, IB, cfg.items, n, tile);
  const int64_t max_s = (n + tile - 1) / tile;
  if (cfg.S > max_s) cfg.S = (int)max_s;
  return cfg;
}

// A launch shape from the ABI's (K, L, T, WG); T, WG = 0 take the defaults.
Launch make_shape(int K, int L, int S, int items, int T, int WG) {
  Launch c{K, L, S, items};
  c.T = T > 0 ? T : nb::kTile;
  c.WG = WG > 0 ? WG : nb::kWG;
  return c;
}

// Shape of the batched force kernel: the last tuned entry of this kind whose
// key range holds `key`, else one i-particle per lane (K = 1) in the LDS
// layout the single-system table gives for a system of the mean size -- a
// block step's active rows are spread over many small systems, and a wider
// i-block would mostly carry empty lanes.
Launch choose_batch(const nb_ctx* c, int kind, int64_t key, int64_t n_total, int64_t mean_size) {
  for (auto it = c->batch_table.rbegin(); it != c->batch_table.rend(); ++it)
    if (it->prec == c->prec && it->kind == kind && key >= it->key_min && key <= it->key_max) return it->cfg;
  Launch cfg = choose(c, n_total, mean_size);
  cfg.K = 1;
  if (cfg.L != 1 && cfg.L != 4 && cfg.L != 16 && cfg.L != 64)
    cfg.L = cfg.L >= 64 ? 64 : cfg.L >= 16 ? 16 : cfg.L >= 4 ? 4 : 1;
  return cfg;
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

bool kernel_mask(int prec, double eps2) {
  return prec == NB_PREC_FP64 ? eps2 == 0.0 : (float)eps2 == 0.0f;
}

// Fixed scratch of the no-allocation entry point: the j-split partials and
// the j-record mirror of one call live here instead of in context memory.
// Each device the library runs on holds its own copy for the life of the
// process.  Host code never uses the array's name as an address: the device
// address is resolved once per device (scratch_address) and passed on.
constexpr size_t kScratchBytes = NB_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices] = {};
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Resolve the device address of `scratch` on `device`, which must be the
// current device; the first call per device does the lookup.
void* scratch_address(int device, hipError_t* err) {
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    g_scratch_ptr[device] = p;
    g_scratch_err[device] = e;
    g_scratch_done[device] = true;
  }
  *err = g_scratch_err[device];
  return g_scratch_ptr[device];
}

// Caller-provided buffers for run_forces: partials and mirror are taken from
// here instead of being grown in the context.
struct FixedScratch {
  double* part;
  void* rec;
};

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int run_forces(nb_ctx* c, const Launch& cfg, const double* pos, const double* vel, const double* mass, int64_t N,
               const int32_t* active, int64_t n_active, double eps2, double* acc, double* jerk, double* pot,
               const double* ipos = nullptr, const double* ivel = nullptr, bool no_self = false,
               const FixedScratch* fixed = nullptr, int64_t n_rows = -1) {
  log_launch(c, "forces", cfg, N, n_active);
  nb::ForceArgs a{};
  a.pos = pos; a.vel = vel; a.mass = mass; a.n = N;
  a.ipos = ipos; a.ivel = ivel; a.no_self = no_self ? 1 : 0;
  a.active = active; a.n_active = n_active; a.n_active_dev = nullptr;
  a.eps2 = eps2; a.S = cfg.S; a.target_items = cfg.items > 0 ? cfg.items : default_items(c, cfg);
  a.acc = acc; a.jerk = jerk; a.pot = pot; a.part = nullptr; a.s_dev = nullptr; a.wq = c->wq;
  a.row_lo = 0; a.row_hi = n_rows >= 0 ? n_rows : N; a.err = c->wq + nb::kErrorWord;
  const bool mask = kernel_mask(c->prec, eps2);
  const Launch eff = mask ? nb::masked(cfg) : cfg;
  const int max_grid = resident_grid(c, eff, mask);
  if (eff.L <= 0) {
    if (fixed) {
      a.rec = fixed->rec;
    } else {
      int rc = ensure_mirror(c, N);
      if (rc) return rc;
      a.rec = c->mirror;
    }
  }
  if (cfg.S > 1 && c->split_atomic && !fixed) {
    if (mask || !nb::atomic_split_supported(eff))
      return fail(c, NB_ENOTSUP, "the atomic j-split sum runs the LDS families 1 and 2 with eps2 > 0 only%s");
    hipError_t e = nb::launch_forces_atomic(c->prec, eff, a, c->stream, max_grid);
    return e == hipSuccess ? NB_OK : hip_fail(c, e, "atomic force launch");
  }
  if (cfg.S > 1) {
    if (fixed) {
      a.part = fixed->part;
    } else {
      const size_t bytes = (size_t)cfg.S * 7 * (size_t)n_active * sizeof(double);
      int rc = ensure_ws(c, bytes);
      if (rc) return rc;
      a.part = static_cast<double*>(c->ws);
    }
  }
  hipError_t e = nb::launch_forces(c->prec, eff, mask, a, c->stream, 0, max_grid);
  if (e != hipSuccess) return hip_fail(c, e, "force kernel launch");
  if (cfg.S > 1) {
    const int IB = nb::ib_of(eff);
    e = nb::launch_reduce_ib(c->prec, a, cfg.S, IB, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reduce kernel launch");
  }
  return NB_OK;
}

int check_forces_args(nb_ctx* c, const double* pos, const double* vel, const double* mass, int64_t N,
                      const void* active, int64_t n_active, double eps2, double* acc, double* jerk, double* pot) {
  if (!c) return NB_EINVAL;
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  if (n_active < 0) return fail(c, NB_EINVAL, "n_active must be >= 0%s");
  if (!finite_nonneg(eps2)) return fail(c, NB_EINVAL, "eps2 must be finite and >= 0%s");
  if (n_active > 0 && (!pos || !vel || !mass || !active || !acc || !jerk || !pot))
    return fail(c, NB_EINVAL, "null pointer argument%s");
  return NB_OK;
}

}  // namespace

extern "C" {

const char* nb_version(void) { return kVersion; }

int nb_create(nb_ctx** out, int device, int precision) {
  if (!out) return NB_EINVAL;
  *out = nullptr;
  if (!valid_prec(precision)) return NB_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return NB_EDEVICE;
  }
  if (device < 0 || device >= ndev) return NB_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return NB_EDEVICE;
  nb_ctx* c = new (std::nothrow) nb_ctx();
  if (!c) return NB_ENOMEM;
  c->device = device;
  c->prec = precision;
  c->log_level = log_level_from_env();
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) == hipSuccess && p.multiProcessorCount > 0) c->num_cus = p.multiProcessorCount;
  // the fixed scratch's address on this device, looked up once per device
  // (a failure is reported by the entry point that needs it)
  hipError_t se = hipSuccess;
  (void)scratch_address(device, &se);
  // the force grids' work queue starts at zero and every launch leaves it
  // at zero
  if (hipMalloc(&c->wq, nb::kWorkQueueWords * sizeof(unsigned int)) != hipSuccess ||
      hipMemset(c->wq, 0, nb::kWorkQueueWords * sizeof(unsigned int)) != hipSuccess) {
    (void)hipGetLastError();
    if (c->wq) (void)hipFree(c->wq);
    delete c;
    return NB_ENOMEM;
  }
  *out = c;
  return NB_OK;
}

int nb_destroy(nb_ctx* c) {
  if (!c) return NB_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->ws) (void)hipFree(c->ws);
  if (c->mirror) (void)hipFree(c->mirror);
  if (c->sched_tmp) (void)hipFree(c->sched_tmp);
  if (c->sched_cnt) (void)hipFree(c->sched_cnt);
  if (c->nact32) (void)hipFree(c->nact32);
  if (c->s_dev) (void)hipFree(c->s_dev);
  if (c->wq) (void)hipFree(c->wq);
  if (c->energy_part) (void)hipFree(c->energy_part);
  if (c->batch_buf) (void)hipFree(c->batch_buf);
  if (c->batch_host) (void)hipHostFree(c->batch_host);
  if (c->batch_ev) (void)hipEventDestroy(c->batch_ev);
  if (c->bp_buf) (void)hipFree(c->bp_buf);
  for (hipEvent_t& ev : c->phase_ev)
    if (ev) (void)hipEventDestroy(ev);
  nb::tree_scratch_free(c->tree);
  delete c;
  return NB_OK;
}

int nb_sync(nb_ctx* c) {
  if (!c) return NB_EINVAL;
  (void)hipSetDevice(c->device);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
  unsigned int words[nb::kWorkQueueWords];
  e = hipMemcpy(words, c->wq, sizeof words, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "reading the device work queue");
  bool queue_dirty = false;
  for (int k = 0; k < nb::kWorkQueueWords; ++k) queue_dirty |= k != nb::kErrorWord && words[k] != 0;
  const unsigned int bits = words[nb::kErrorWord];
  if (!bits && !queue_dirty) return NB_OK;
  // clear everything, so the calls after this one start from a clean queue
  e = hipMemsetAsync(c->wq, 0, sizeof words, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "clearing the device work queue");
  if (bits & nb::kErrTreeStack)
    return fail(c, NB_ENOMEM, "a tree walk's stack reached its bound since the last nb_sync; its groups' forces "
                              "were not written%s");
  if (queue_dirty)
    return fail(c, NB_EINVAL,
                "the work-queue counters were not zero after synchronising: calls on this context overlapped on "
                "the device (another stream, or a graph replayed on another stream); results since the last "
                "nb_sync cannot be trusted%s");
  return fail(c, NB_EINVAL,
              "an active_idx entry outside its valid range was passed since the last nb_sync; its rows were "
              "skipped (outputs not written)%s");
}

int nb_check_active_host(const int32_t* active, int64_t n_active, int64_t lo, int64_t hi, int64_t* first_bad) {
  if (n_active < 0 || (n_active > 0 && !active)) return NB_EINVAL;
  for (int64_t k = 0; k < n_active; ++k)
    if (!nb::row_in_range(active[k], lo, hi)) {
      if (first_bad) *first_bad = k;
      return NB_EINVAL;
    }
  if (first_bad) *first_bad = -1;
  return NB_OK;
}

int nb_workspace_bytes(const nb_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return NB_EINVAL;
  *bytes = (int64_t)(c->ws_bytes + c->mirror_bytes);
  return NB_OK;
}

int nb_set_stream(nb_ctx* c, void* s) {
  if (!c) return NB_EINVAL;
  c->stream = static_cast<hipStream_t>(s);
  return NB_OK;
}

int nb_set_precision(nb_ctx* c, int precision) {
  if (!c) return NB_EINVAL;
  if (!valid_prec(precision)) return fail(c, NB_EINVAL, "unknown precision%s");
  c->prec = precision;
  return NB_OK;
}

int nb_get_precision(const nb_ctx* c) { return c ? c->prec : NB_EINVAL; }

const char* nb_last_error(const nb_ctx* c) { return c ? c->err.c_str() : "null context"; }

int nb_set_launch(nb_ctx* c, int K, int L, int S, int T, int WG) {
  if (!c) return NB_EINVAL;
  if (K == 0) {
    c->have_forced = false;
    return NB_OK;
  }
  if (!valid_K(K) || !valid_L(L) || S < 0 || T < 0 || WG < 0) return fail(c, NB_EINVAL, "bad launch configuration%s");
  if (!nb::launch_supported(make_shape(K, L, 1, 0, T, WG))) return fail(c, NB_ENOTSUP, "launch shape not built%s");
  c->forced = make_shape(K, L, S, 0, T, WG);
  c->have_forced = true;
  return NB_OK;
}

int nb_get_launch(nb_ctx* c, int64_t N, int64_t n_active, int* K, int* L, int* S, int* T, int* WG) {
  if (!c || !K || !L || !S || N < 1 || n_active < 0) return NB_EINVAL;
  const Launch cfg = choose(c, N, n_active < 1 ? 1 : n_active);
  *K = cfg.K; *L = cfg.L; *S = cfg.S;
  if (T) *T = cfg.T;
  if (WG) *WG = cfg.WG;
  return NB_OK;
}

int nb_tune_add(nb_ctx* c, int precision, int64_t n_min, int64_t act_min, int64_t act_max, int K, int L, int S,
                int T, int WG) {  // S: work-item target
  if (!c) return NB_EINVAL;
  if (!valid_prec(precision) || !valid_K(K) || !valid_L(L) || S < 0 || T < 0 || WG < 0 || act_min > act_max)
    return fail(c, NB_EINVAL, "bad tune entry%s");
  if (!nb::launch_supported(make_shape(K, L, 1, 0, T, WG))) return fail(c, NB_ENOTSUP, "launch shape not built%s");
  c->table.push_back(nb::TuneEntry{precision, n_min, act_min, act_max, make_shape(K, L, 0, S, T, WG)});
  return NB_OK;
}

int nb_set_split_sum(nb_ctx* c, int mode) {
  if (!c) return NB_EINVAL;
  if (mode != 0 && mode != 1) return fail(c, NB_EINVAL, "split-sum mode must be 0 (fixed order) or 1 (atomic)%s");
  c->split_atomic = mode == 1;
  return NB_OK;
}

int nb_tune_add_batch(nb_ctx* c, int precision, int kind, int64_t key_min, int64_t key_max, int K, int L) {
  if (!c) return NB_EINVAL;
  if (!valid_prec(precision) || (kind != 1 && kind != 2) || key_min > key_max || !valid_K(K) || L < 0)
    return fail(c, NB_EINVAL, "bad batch tune entry%s");
  if (!nb::batch_supported(Launch{K, L, 1})) return fail(c, NB_ENOTSUP, "batched kernel not built in this shape%s");
  c->batch_table.push_back(nb::BatchTuneEntry{precision, kind, key_min, key_max, Launch{K, L, 0, 0}});
  return NB_OK;
}

int nb_get_batch_launch(nb_ctx* c, int kind, int64_t key, int64_t n_total, int* K, int* L) {
  if (!c || !K || !L || (kind != 1 && kind != 2) || n_total < 1 || key < 1) return NB_EINVAL;
  const Launch cfg = choose_batch(c, kind, key, n_total, key);
  *K = cfg.K;
  *L = cfg.L;
  return NB_OK;
}

int nb_set_stop_source(nb_ctx* c, const int64_t* t_stop_dev) {
  if (!c) return NB_EINVAL;
  c->stop_dev = t_stop_dev;
  return NB_OK;
}

int nb_set_phase_timing(nb_ctx* c, int on) {
  if (!c) return NB_EINVAL;
  if (on && !c->phase_ev[0]) {
    (void)hipSetDevice(c->device);
    for (hipEvent_t& ev : c->phase_ev) {
      if (hipEventCreate(&ev) != hipSuccess) {
        const hipError_t e = hipGetLastError();
        for (hipEvent_t& f : c->phase_ev) {
          if (f) (void)hipEventDestroy(f);
          f = nullptr;
        }
        return hip_fail(c, e, "phase timing events");
      }
    }
  }
  c->phase_on = on != 0;
  c->phase_valid = false;
  return NB_OK;
}

int nb_phase_times(nb_ctx* c, float ms[3]) {
  if (!c || !ms) return NB_EINVAL;
  if (!c->phase_on || !c->phase_valid)
    return fail(c, NB_EINVAL, "no eager block step was timed since phase timing was switched on%s");
  hipError_t e = hipEventSynchronize(c->phase_ev[3]);
  if (e != hipSuccess) return hip_fail(c, e, "phase timing wait");
  for (int k = 0; k < 3; ++k) {
    e = hipEventElapsedTime(&ms[k], c->phase_ev[k], c->phase_ev[k + 1]);
    if (e != hipSuccess) return hip_fail(c, e, "phase timing");
  }
  return NB_OK;
}

int nb_tune_clear(nb_ctx* c) {
  if (!c) return NB_EINVAL;
  c->table.clear();
  c->batch_table.clear();
  return NB_OK;
}

int nbody_forces(nb_ctx* c, const double* pos, const double* vel, const double* mass, int64_t N,
                 const int32_t* active, int64_t n_active, double eps2, double* acc, double* jerk, double* pot) {
  int rc = check_forces_args(c, pos, vel, mass, N, active, n_active, eps2, acc, jerk, pot);
  if (rc) return rc;
  if (n_active == 0) return NB_OK;
  const Launch cfg = choose(c, N, n_active);
  return run_forces(c, cfg, pos, vel, mass, N, active, n_active, eps2, acc, jerk, pot);
}

int nbody_forces_noalloc(nb_ctx* c, const double* pos, const double* vel, const double* mass, int64_t N,
                         const int32_t* active, int64_t n_active, double eps2, double* acc, double* jerk,
                         double* pot) {
  int rc = check_forces_args(c, pos, vel, mass, N, active, n_active, eps2, acc, jerk, pot);
  if (rc) return rc;
  if (n_active == 0) return NB_OK;
  hipError_t se = hipSuccess;
  unsigned char* base = static_cast<unsigned char*>(scratch_address(c->device, &se));
  if (!base) return hip_fail(c, se, "address of the fixed scratch");
  // the launch nbody_forces would take, so the two give identical results
  Launch cfg = choose(c, N, n_active);
  const size_t row_bytes = 7 * sizeof(double) * (size_t)n_active;  // one j-chunk's partial sums
  auto part_bytes = [&](int S) { return S > 1 ? align256((size_t)S * row_bytes) : (size_t)0; };
  const size_t rec = cfg.L <= 0 ? nb::mirror_bytes(c->prec, N) : 0;
  if (part_bytes(cfg.S) + rec > kScratchBytes) {
    // an automatic launch takes the largest j-split whose partials fit (the
    // sums then differ from nbody_forces only in their order); a forced
    // launch, or a mirror that alone does not fit, is refused
    const size_t avail = rec < kScratchBytes ? kScratchBytes - rec : 0;
    const int64_t s_fit = avail > 255 ? (int64_t)((avail - 255) / row_bytes) : 0;
    if (c->have_forced || rec > kScratchBytes) {
      char buf[256];
      std::snprintf(buf, sizeof buf,
                    "launch (K=%d, L=%d, S=%d) needs %zu bytes of scratch, more than the fixed %zu; "
                    "use nbody_forces, or a smaller S through nb_set_launch",
                    cfg.K, cfg.L, cfg.S, part_bytes(cfg.S) + rec, kScratchBytes);
      c->err = buf;
      return NB_ENOMEM;
    }
    cfg.S = s_fit >= 2 ? (int)std::min<int64_t>(s_fit, cfg.S) : 1;
  }
  const size_t part = part_bytes(cfg.S);
  const FixedScratch fx{reinterpret_cast<double*>(base), rec ? base + part : nullptr};
  return run_forces(c, cfg, pos, vel, mass, N, active, n_active, eps2, acc, jerk, pot, nullptr, nullptr, false,
                    &fx);
}

int nbody_forces_ij(nb_ctx* c, const double* pos_j, const double* vel_j, const double* mass_j, int64_t N_j,
                    const double* pos_i, const double* vel_i, int64_t N_i, const int32_t* active, int64_t n_active,
                    double eps2, double* acc, double* jerk, double* pot) {
  int rc = check_forces_args(c, pos_j, vel_j, mass_j, N_j, active, n_active, eps2, acc, jerk, pot);
  if (rc) return rc;
  if (N_i < 0 || N_i >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N_i must be in [0, 2^31)%s");
  if (n_active > 0 && (N_i < 1 || !pos_i || !vel_i))
    return fail(c, NB_EINVAL, "i-particle arrays are empty or null%s");
  if (n_active == 0) return NB_OK;
  const Launch cfg = choose(c, N_j, n_active);
  return run_forces(c, cfg, pos_j, vel_j, mass_j, N_j, active, n_active, eps2, acc, jerk, pot, pos_i, vel_i, true,
                    nullptr, N_i);
}

int nb_time_forces(nb_ctx* c, int K, int L, int S, int T, int WG, const double* pos, const double* vel,
                   const double* mass, int64_t N, const int32_t* active, int64_t n_active, double eps2, double* acc,
                   double* jerk, double* pot, int reps, double* ms) {
  int rc = check_forces_args(c, pos, vel, mass, N, active, n_active, eps2, acc, jerk, pot);
  if (rc) return rc;
  if (!ms || reps < 1 || n_active < 1) return fail(c, NB_EINVAL, "reps >= 1, n_active >= 1 and ms required%s");
  if (!valid_K(K) || !valid_L(L) || S < 0 || T < 0 || WG < 0) return fail(c, NB_EINVAL, "bad launch configuration%s");
  Launch cfg = make_shape(K, L, S, 0, T, WG);
  if (!nb::launch_supported(make_shape(K, L, 1, 0, T, WG))) return fail(c, NB_ENOTSUP, "launch shape not built%s");
  if (kernel_mask(c->prec, eps2) && !nb::default_tile(cfg))
    return fail(c, NB_ENOTSUP, "eps2 = 0 runs the default tile and workgroup size only%s");
  cfg.items = default_items(c, cfg);
  const int tile = cfg.L > 0 ? cfg.T : nb::kTile;
  if (cfg.S == 0) cfg.S = nb::host_choose_S(n_active, nb::ib_of(cfg), cfg.items, N, tile);
  const int64_t max_s = (N + tile - 1) / tile;
  if (cfg.S > max_s) cfg.S = (int)max_s;
  rc = run_forces(c, cfg, pos, vel, mass, N, active, n_active, eps2, acc, jerk, pot);
  if (rc) return rc;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return hip_fail(c, hipGetLastError(), "hipEventCreate");
  (void)hipEventRecord(e0, c->stream);
  for (int r = 0; r < reps && rc == NB_OK; ++r)
    rc = run_forces(c, cfg, pos, vel, mass, N, active, n_active, eps2, acc, jerk, pot);
  (void)hipEventRecord(e1, c->stream);
  hipError_t e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(c, e, "timing");
  *ms = (double)t / reps;
  return NB_OK;
}

// Device-count variant: the active count lives in device memory, so the
// launch configuration is fixed per regime of the count and each regime's
// kernels return at once when the count is outside it.  Every regime's
// workspace need is bounded on the host from max_active.
}  // extern "C"

namespace {

// The device-count force launches; with `reduce` also the shared reduce,
// otherwise its arguments go to *red for a caller that fuses it with the
// next pass (the block step).
int devcount_forces(nb_ctx* c, const double* pos, const double* vel, const double* mass, int64_t N,
                    const int32_t* active, const int32_t* n_active_dev, int64_t max_active, double eps2,
                    double* acc, double* jerk, double* pot, bool reduce, nb::ForceArgs* red_out) {
  int rc = check_forces_args(c, pos, vel, mass, N, active, max_active, eps2, acc, jerk, pot);
  if (rc) return rc;
  if (!n_active_dev) return fail(c, NB_EINVAL, "n_active_dev is null%s");
  if (max_active == 0) return NB_OK;
  const bool mask = kernel_mask(c->prec, eps2);
  // One fixed launch per group of regimes; the count decides on the device
  // which one works.  Every launch, empty or not, costs a few microseconds
  // in each block step, so adjacent regimes share a launch: those of one
  // shape, and LDS regimes of different shapes that one kernel family holds
  // (family_of).  A family kernel has the registers of its largest body, so
  // a regime joins one only when it loses nothing: its whole grid fits in
  // one round of the family's resident workgroups, or the family keeps as
  // many resident as the regime's own kernel.  The shared launch carries
  // each regime's shape and work-item target, so a count gets the shape and
  // j-split of a host-count launch.
  struct Group {
    Regime r;   // merged count range; r.cfg: the shape of the first regime (fam set for a family launch)
    int n_sub;
    int64_t sub_lo[nb::kMaxSubRegimes];
    int64_t sub_hi[nb::kMaxSubRegimes];
    int sub_items[nb::kMaxSubRegimes];
    int64_t sub_grid[nb::kMaxSubRegimes];  // workgroups the regime can use
    Launch sub_cfg[nb::kMaxSubRegimes];
  };
  auto fam_of = [](const Launch& x) { return x.L >= 1 && nb::default_tile(x) ? nb::family_of(x.K, x.L) : 0; };
  auto own_rg = [&](const Launch& x) {
    Launch o = x;
    o.fam = fam_of(x);
    return resident_grid(c, o, mask);
  };
  std::vector<Group> groups;
  for (const Regime& r : regimes(c, N)) {
    Launch cfg = c->have_forced ? c->forced : r.cfg;
    if (mask) cfg = nb::masked(cfg);
    cfg.fam = 0;
    const int items = cfg.items > 0 ? cfg.items : default_items(c, cfg);
    const int64_t top = r.hi < max_active ? r.hi : max_active;
    const int IB = nb::ib_of(cfg);
    const int64_t grid = items + (top > 0 ? (top + IB - 1) / IB : 0);
    bool join = false;
    int fam = 0;
    if (!groups.empty() && groups.back().n_sub < nb::kMaxSubRegimes) {
      const Group& g = groups.back();
      if (g.r.cfg.fam == 0 && g.r.cfg.K == cfg.K && g.r.cfg.L == cfg.L && g.r.cfg.T == cfg.T &&
          g.r.cfg.WG == cfg.WG) {
        join = true;
      } else if (cfg.L >= 1 && g.r.cfg.L >= 1) {
        const int theirs = g.r.cfg.fam > 0 ? g.r.cfg.fam : fam_of(g.r.cfg);
        fam = nb::family_cover(theirs, fam_of(cfg));
        if (fam) {
          Launch fcfg = cfg;
          fcfg.fam = fam;
          const int64_t frg = resident_grid(c, fcfg, mask);
          join = grid <= frg || frg >= own_rg(cfg);
          for (int k = 0; join && k < g.n_sub; ++k)
            join = g.sub_grid[k] <= frg || frg >= own_rg(g.sub_cfg[k]);
        }
      }
    }
    if (join) {
      Group& g = groups.back();
      if (fam) g.r.cfg.fam = fam;
      g.r.hi = r.hi;
      g.sub_lo[g.n_sub] = r.lo;
      g.sub_hi[g.n_sub] = r.hi;
      g.sub_items[g.n_sub] = items;
      g.sub_grid[g.n_sub] = grid;
      g.sub_cfg[g.n_sub] = cfg;
      ++g.n_sub;
    } else {
      Group g{};
      g.r = r;
      g.r.cfg = cfg;
      g.n_sub = 1;
      g.sub_lo[0] = r.lo;
      g.sub_hi[0] = r.hi;
      g.sub_items[0] = items;
      g.sub_grid[0] = grid;
      g.sub_cfg[0] = cfg;
      groups.push_back(g);
    }
  }
  // per regime of a group: the rows of its partials and its part of the grid
  auto sub_top = [&](const Group& g, int k) { return g.sub_hi[k] < max_active ? g.sub_hi[k] : max_active; };
  size_t ws_need = 0;
  for (const Group& g : groups) {
    if (g.r.lo > max_active) break;
    for (int k = 0; k < g.n_sub; ++k) {
      if (g.sub_lo[k] > max_active) break;
      const int IB = nb::ib_of(g.sub_cfg[k]);
      const int64_t n_iblk_max = (sub_top(g, k) + IB - 1) / IB;
      const size_t rows = (size_t)(g.sub_items[k] + n_iblk_max) * IB;
      const size_t need = rows * 7 * sizeof(double);
      if (need > ws_need) ws_need = need;
    }
  }
  rc = ensure_ws(c, ws_need);
  if (rc) return rc;
  bool need_mirror = false;
  for (const Group& g : groups)
    if (g.r.lo <= max_active && (c->have_forced ? c->forced.L : g.r.cfg.L) <= 0) need_mirror = true;
  if (need_mirror) {
    rc = ensure_mirror(c, N);
    if (rc) return rc;
  }
  if (!c->s_dev) {
    if (capturing(c->stream)) return fail(c, NB_ENOMEM, "the split slot must be allocated before capture%s");
    if (hipMalloc(&c->s_dev, sizeof(int)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, NB_ENOMEM, "hipMalloc of the split slot failed%s");
    }
  }
  nb::ForceArgs red{};
  for (const Group& g : groups) {
    if (g.r.lo > max_active) break;
    const int64_t top = g.r.hi < max_active ? g.r.hi : max_active;
    Launch cfg = c->have_forced ? c->forced : g.r.cfg;
    if (mask) cfg = nb::masked(cfg);
    if (c->log_level >= 2) {
      std::fprintf(stderr, "nbody: count-on-device launch for n_active in [%lld, %lld], family %d:\n",
                   (long long)g.r.lo, (long long)top, g.r.cfg.fam);
      for (int k = 0; k < g.n_sub && g.sub_lo[k] <= max_active; ++k)
        log_launch(c, "  regime", g.sub_cfg[k], N, g.sub_lo[k]);
    }
    nb::ForceArgs a{};
    a.pos = pos; a.vel = vel; a.mass = mass; a.n = N;
    a.active = active; a.n_active = top; a.n_active_dev = n_active_dev;
    a.act_lo = g.r.lo;
    a.last = (top == max_active) ? 1 : 0;
    a.eps2 = eps2; a.S = 1; a.target_items = g.sub_items[0];
    a.n_sub = g.n_sub;
    // persistent: at most one round of resident workgroups walks the items
    int64_t grid = 1;
    for (int k = 0; k < g.n_sub; ++k) {
      a.sub_lo[k] = g.sub_lo[k];
      a.sub_items[k] = g.sub_items[k];
      a.sub_shape[k] = nb::shape_code(g.sub_cfg[k].K, g.sub_cfg[k].L);
      if (g.sub_lo[k] > max_active) continue;
      const int IB = nb::ib_of(g.sub_cfg[k]);
      grid = std::max<int64_t>(grid, g.sub_items[k] + (sub_top(g, k) + IB - 1) / IB);
    }
    a.shape = a.sub_shape[0];
    a.acc = acc; a.jerk = jerk; a.pot = pot; a.part = static_cast<double*>(c->ws); a.s_dev = c->s_dev;
    a.rec = c->mirror;
    a.wq = c->wq;
    a.row_lo = 0; a.row_hi = N; a.err = c->wq + nb::kErrorWord;
    red = a;
    const int64_t rg = resident_grid(c, cfg, mask);
    if (grid > rg) grid = rg;
    hipError_t e = nb::launch_forces(c->prec, cfg, mask, a, c->stream, (int)grid, 0);
    if (e != hipSuccess) return hip_fail(c, e, "force kernel launch (device count)");
  }
  // one reduce for all regimes: the regime that worked left its S in s_dev
  red.n_active = max_active;
  red.act_lo = 0;
  red.last = 1;
  if (red_out) *red_out = red;
  if (!reduce) return NB_OK;
  hipError_t e = nb::launch_reduce_ib(c->prec, red, 1, 1, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "reduce kernel launch (device count)");
  return NB_OK;
}

}  // namespace

extern "C" {

int nbody_forces_devcount(nb_ctx* c, const double* pos, const double* vel, const double* mass, int64_t N,
                          const int32_t* active, const int32_t* n_active_dev, int64_t max_active, double eps2,
                          double* acc, double* jerk, double* pot) {
  return devcount_forces(c, pos, vel, mass, N, active, n_active_dev, max_active, eps2, acc, jerk, pot, true,
                         nullptr);
}

int hermite_predict(nb_ctx* c, const double* pos, const double* vel, const double* acc, const double* jerk,
                    const int64_t* t_tick, int64_t t_next_tick, double dt_min, int64_t N, double* pos_p,
                    double* vel_p) {
  if (!c) return NB_EINVAL;
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  if (!pos || !vel || !acc || !jerk || !t_tick || !pos_p || !vel_p) return fail(c, NB_EINVAL, "null pointer%s");
  if (!(dt_min > 0.0) || !std::isfinite(dt_min)) return fail(c, NB_EINVAL, "dt_min must be finite and > 0%s");
  hipError_t e = nb::launch_predict(pos, vel, acc, jerk, t_tick, t_next_tick, nullptr, dt_min, N, pos_p, vel_p,
                                    c->stream);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, "predict launch");
}

// ---- sixth-order Hermite ---------------------------------------------------
static int run_forces6(nb_ctx* c, const double* pos, const double* vel, const double* accj, const double* mass,
                       int64_t N, const int32_t* active, int64_t n_max, const int32_t* n_active_dev, double eps2,
                       double* acc, double* jerk, double* snap, double* pot) {
  const bool mask = eps2 == 0.0;
  const int grid = c->num_cus * nb::forces6_resident_wgs(mask);
  const int target = 4 * grid;
  nb::Force6Args a{};
  a.pos = pos; a.vel = vel; a.accj = accj; a.mass = mass; a.n = N;
  a.active = active; a.n_active = n_max; a.n_active_dev = n_active_dev; a.eps2 = eps2;
  a.target_items = target;
  a.S = nb::forces6_split(n_max, target, N);
  a.acc = acc; a.jerk = jerk; a.snap = snap; a.pot = pot;
  a.err = c->wq + nb::kErrorWord;
  const int64_t rows = n_active_dev ? nb::forces6_workspace_rows(n_max, target, N) : (int64_t)a.S * n_max;
  if (n_active_dev || a.S > 1) {
    int rc = ensure_ws(c, (size_t)rows * 10 * sizeof(double));
    if (rc) return rc;
    a.part = static_cast<double*>(c->ws);
  }
  hipError_t e = nb::launch_forces6(a, mask, grid, c->stream);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, "sixth-order force launch");
}

int nbody_forces6(nb_ctx* c, const double* pos, const double* vel, const double* acc_j, const double* mass, int64_t N,
                  const int32_t* active, int64_t n_active, double eps2, double* acc, double* jerk, double* snap,
                  double* pot) {
  int rc = check_forces_args(c, pos, vel, mass, N, active, n_active, eps2, acc, jerk, pot);
  if (rc) return rc;
  if (n_active > 0 && (!acc_j || !snap)) return fail(c, NB_EINVAL, "null pointer argument%s");
  if (n_active == 0) return NB_OK;
  return run_forces6(c, pos, vel, acc_j, mass, N, active, n_active, nullptr, eps2, acc, jerk, snap, pot);
}

int hermite6_predict(nb_ctx* c, const double* pos, const double* vel, const double* acc, const double* jerk,
                     const double* snap, const double* crackle, const int64_t* t_tick, int64_t t_next_tick,
                     double dt_min, int64_t N, double* pos_p, double* vel_p, double* acc_p) {
  if (!c) return NB_EINVAL;
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  if (!pos || !vel || !acc || !jerk || !snap || !crackle || !t_tick || !pos_p || !vel_p || !acc_p)
    return fail(c, NB_EINVAL, "null pointer%s");
  if (!(dt_min > 0.0) || !std::isfinite(dt_min)) return fail(c, NB_EINVAL, "dt_min must be finite and > 0%s");
  hipError_t e = nb::launch_predict6(pos, vel, acc, jerk, snap, crackle, t_tick, t_next_tick, nullptr, dt_min, N,
                                     pos_p, vel_p, acc_p, c->stream);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, "sixth-order predict launch");
}

static int check_levels(nb_ctx* c, double eta, double dt_max, int32_t max_level);

int hermite6_correct(nb_ctx* c, const int32_t* active, int64_t n_active, int64_t N, const double* acc1,
                     const double* jerk1,
                     const double* snap1, double* pos, double* vel, double* acc, double* jerk, double* snap,
                     double* crackle, int64_t* t_tick, int32_t* dt_level, double eta, double dt_max,
                     int32_t max_level, int64_t* clamp_count_dev) {
  if (!c) return NB_EINVAL;
  if (n_active < 0 || n_active >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "n_active must be in [0, 2^31)%s");
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  int rc = check_levels(c, eta, dt_max, max_level);
  if (rc) return rc;
  if (n_active == 0) return NB_OK;
  if (!active || !acc1 || !jerk1 || !snap1 || !pos || !vel || !acc || !jerk || !snap || !crackle || !t_tick ||
      !dt_level)
    return fail(c, NB_EINVAL, "null pointer%s");
  hipError_t e = nb::launch_correct6(active, n_active, nullptr, N, c->wq + nb::kErrorWord, acc1, jerk1, snap1, pos, vel, acc,
                                     jerk, snap,
                                     crackle, t_tick, dt_level, eta, dt_max, max_level, clamp_count_dev, nullptr,
                                     c->stream);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, "sixth-order correct launch");
}

int hermite6_startup(nb_ctx* c, const double* acc, const double* jerk, const double* snap, int64_t N, double eta_s,
                     double dt_max, int32_t max_level, int32_t* dt_level) {
  if (!c) return NB_EINVAL;
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  int rc = check_levels(c, eta_s, dt_max, max_level);
  if (rc) return rc;
  if (!acc || !jerk || !snap || !dt_level) return fail(c, NB_EINVAL, "null pointer%s");
  hipError_t e = nb::launch_startup6(acc, jerk, snap, N, eta_s, dt_max, max_level, dt_level, c->stream);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, "sixth-order startup launch");
}

int nb_block_step6(nb_ctx* c, int64_t N, double eps2, double eta, double dt_max, int32_t max_level,
                   const double* mass, double* pos, double* vel, double* acc, double* jerk, double* snap,
                   double* crackle, int64_t* t_tick, int32_t* dt_level, double* pos_p, double* vel_p, double* acc_p,
                   int32_t* active, double* acc1, double* jerk1, double* snap1, double* pot1, int64_t* sched,
                   int64_t t_stop_tick) {
  if (!c) return NB_EINVAL;
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  int rc = check_levels(c, eta, dt_max, max_level);
  if (rc) return rc;
  if (!finite_nonneg(eps2)) return fail(c, NB_EINVAL, "eps2 must be finite and >= 0%s");
  if (!mass || !pos || !vel || !acc || !jerk || !snap || !crackle || !t_tick || !dt_level || !pos_p || !vel_p ||
      !acc_p || !active || !acc1 || !jerk1 || !snap1 || !pot1 || !sched)
    return fail(c, NB_EINVAL, "null pointer%s");
  rc = ensure_sched(c, N);
  if (rc) return rc;
  const double dt_min = std::ldexp(dt_max, -max_level);
  phase_mark(c, 0);
  hipError_t e = nb::launch_schedule(t_tick, dt_level, N, max_level, active, sched, c->sched_tmp, c->sched_cnt,
                                     c->nact32, t_stop_tick, c->stop_dev, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "schedule launch");
  e = nb::launch_predict6(pos, vel, acc, jerk, snap, crackle, t_tick, 0, sched, dt_min, N, pos_p, vel_p, acc_p,
                          c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "sixth-order predict launch");
  phase_mark(c, 1);
  rc = run_forces6(c, pos_p, vel_p, acc_p, mass, N, active, N, c->nact32, eps2, acc1, jerk1, snap1, pot1);
  if (rc) return rc;
  phase_mark(c, 2);
  e = nb::launch_correct6(active, N, sched + 1, N, c->wq + nb::kErrorWord, acc1, jerk1, snap1, pos, vel, acc, jerk, snap,
                          crackle, t_tick,
                          dt_level, eta, dt_max, max_level, sched + 3, sched + 2, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "sixth-order correct launch");
  phase_mark(c, 3);
  return NB_OK;
}

// ---- tree code -------------------------------------------------------------
int nb_tree_forces(nb_ctx* c, const double* pos, const double* mass, int64_t N, double eps2, double theta,
                   int32_t n_crit, double g_frac, double* acc, double* pot, int64_t* stats) {
  if (!c) return NB_EINVAL;
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  if (!finite_nonneg(eps2)) return fail(c, NB_EINVAL, "eps2 must be finite and >= 0%s");
  if (!finite_nonneg(theta)) return fail(c, NB_EINVAL, "theta must be finite and >= 0%s");
  if (n_crit < 1) return fail(c, NB_EINVAL, "n_crit must be >= 1%s");
  if (!std::isfinite(g_frac)) return fail(c, NB_EINVAL, "g_frac must be finite%s");
  if (!pos || !mass || !acc || !pot) return fail(c, NB_EINVAL, "null pointer%s");
  const bool cap = capturing(c->stream);
  if (cap && stats) return fail(c, NB_ENOTSUP, "stats need a synchronisation: pass NULL under stream capture%s");
  const char* msg = "";
  nb::TreeStats st{};
  hipError_t e = nb::tree_forces_run(c->tree, c->stream, pos, mass, (int32_t)N, eps2, theta, n_crit, g_frac,
                                     c->prec != NB_PREC_FP64, acc, pot, stats ? &st : nullptr, cap,
                                     c->wq + nb::kErrorWord, &msg);
  if (e == hipErrorStreamCaptureUnsupported)
    return fail(c, NB_ENOTSUP, "the tree buffers must grow: call once outside the capture with this N first%s");
  if (e == hipErrorInvalidValue) return fail(c, NB_ENOMEM, "%s", msg);
  if (e != hipSuccess) return hip_fail(c, e, msg);
  if (stats) {
    stats[0] = st.cells;
    stats[1] = st.groups;
    stats[2] = st.accepted;
    stats[3] = st.opened_leaves;
    stats[4] = st.depth;
  }
  return NB_OK;
}

int nb_tree_keys(nb_ctx* c, const double* pos, int64_t N, uint64_t* keys, int32_t* idx) {
  if (!c) return NB_EINVAL;
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  if (!pos || !keys || !idx) return fail(c, NB_EINVAL, "null pointer%s");
  if (capturing(c->stream)) return fail(c, NB_ENOTSUP, "nb_tree_keys cannot be captured%s");
  const char* msg = "";
  hipError_t e = nb::tree_sorted_keys(c->tree, c->stream, pos, (int32_t)N, keys, idx, &msg);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, msg);
}

int nb_kick(nb_ctx* c, double* vel, const double* acc, int64_t N, double h) {
  if (!c) return NB_EINVAL;
  if (N < 0 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [0, 2^31)%s");
  if (!std::isfinite(h)) return fail(c, NB_EINVAL, "h must be finite%s");
  if (N == 0) return NB_OK;
  if (!vel || !acc) return fail(c, NB_EINVAL, "null pointer%s");
  hipError_t e = nb::launch_kick(vel, acc, h, N, c->stream);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, "kick launch");
}

int nb_kick_drift(nb_ctx* c, double* pos, double* vel, const double* acc, int64_t N, double h_kick, double h_drift) {
  if (!c) return NB_EINVAL;
  if (N < 0 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [0, 2^31)%s");
  if (!std::isfinite(h_kick) || !std::isfinite(h_drift)) return fail(c, NB_EINVAL, "h must be finite%s");
  if (N == 0) return NB_OK;
  if (!pos || !vel || !acc) return fail(c, NB_EINVAL, "null pointer%s");
  hipError_t e = nb::launch_kick_drift(pos, vel, acc, h_kick, h_drift, N, c->stream);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, "kick-drift launch");
}

static int check_levels(nb_ctx* c, double eta, double dt_max, int32_t max_level) {
  if (!(eta > 0.0) || !std::isfinite(eta)) return fail(c, NB_EINVAL, "eta must be finite and > 0%s");
  if (!(dt_max > 0.0) || !std::isfinite(dt_max)) return fail(c, NB_EINVAL, "dt_max must be finite and > 0%s");
  if (max_level < 0 || max_level > 62) return fail(c, NB_EINVAL, "max_level must be in [0, 62]%s");
  return NB_OK;
}

int hermite_correct(nb_ctx* c, const int32_t* active, int64_t n_active, int64_t N, const double* pos_p,
                    const double* vel_p,
                    const double* acc1, const double* jerk1, double* pos, double* vel, double* acc, double* jerk,
                    int64_t* t_tick, int32_t* dt_level, double eta, double dt_max, int32_t max_level,
                    int64_t* clamp_count_dev) {
  if (!c) return NB_EINVAL;
  if (n_active < 0 || n_active >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "bad n_active%s");
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  int rc = check_levels(c, eta, dt_max, max_level);
  if (rc) return rc;
  if (n_active == 0) return NB_OK;
  if (!active || !pos_p || !vel_p || !acc1 || !jerk1 || !pos || !vel || !acc || !jerk || !t_tick || !dt_level)
    return fail(c, NB_EINVAL, "null pointer%s");
  hipError_t e = nb::launch_correct(active, n_active, nullptr, N, c->wq + nb::kErrorWord, pos_p, vel_p, acc1, jerk1, pos, vel,
                                    acc, jerk,
                                    t_tick, dt_level, eta, dt_max, max_level, clamp_count_dev, c->stream);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, "correct launch");
}

int hermite_startup(nb_ctx* c, const double* acc, const double* jerk, int64_t N, double eta, double dt_max,
                    int32_t max_level, int32_t* dt_level) {
  if (!c) return NB_EINVAL;
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  int rc = check_levels(c, eta, dt_max, max_level);
  if (rc) return rc;
  if (!acc || !jerk || !dt_level) return fail(c, NB_EINVAL, "null pointer%s");
  hipError_t e = nb::launch_startup(acc, jerk, N, eta, dt_max, max_level, dt_level, c->stream);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, "startup launch");
}

int nb_schedule(nb_ctx* c, const int64_t* t_tick, const int32_t* dt_level, int64_t N, int32_t max_level,
                int32_t* active, int64_t* sched) {
  if (!c) return NB_EINVAL;
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  if (max_level < 0 || max_level > 62) return fail(c, NB_EINVAL, "max_level must be in [0, 62]%s");
  if (!t_tick || !dt_level || !active || !sched) return fail(c, NB_EINVAL, "null pointer%s");
  int rc = ensure_sched(c, N);
  if (rc) return rc;
  hipError_t e = nb::launch_schedule(t_tick, dt_level, N, max_level, active, sched, c->sched_tmp, c->sched_cnt,
                                     c->nact32, INT64_MAX, nullptr, c->stream);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, "schedule launch");
}

int nb_block_step(nb_ctx* c, int64_t N, double eps2, double eta, double dt_max, int32_t max_level,
                  const double* mass, double* pos, double* vel, double* acc, double* jerk, int64_t* t_tick,
                  int32_t* dt_level, double* pos_p, double* vel_p, int32_t* active, double* acc1, double* jerk1,
                  double* pot1, int64_t* sched, int64_t t_stop_tick) {
  if (!c) return NB_EINVAL;
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  int rc = check_levels(c, eta, dt_max, max_level);
  if (rc) return rc;
  if (!finite_nonneg(eps2)) return fail(c, NB_EINVAL, "eps2 must be finite and >= 0%s");
  if (!mass || !pos || !vel || !acc || !jerk || !t_tick || !dt_level || !pos_p || !vel_p || !active || !acc1 ||
      !jerk1 || !pot1 || !sched)
    return fail(c, NB_EINVAL, "null pointer%s");
  rc = ensure_sched(c, N);
  if (rc) return rc;
  const double dt_min = std::ldexp(dt_max, -max_level);
  phase_mark(c, 0);
  // schedule and predict (the predictor runs in the scheduler's last pass)
  const nb::PredictArgs pred{pos, vel, acc, jerk, dt_min, pos_p, vel_p};
  hipError_t e = nb::launch_schedule(t_tick, dt_level, N, max_level, active, sched, c->sched_tmp, c->sched_cnt,
                                     c->nact32, t_stop_tick, c->stop_dev, c->stream, &pred);
  if (e != hipSuccess) return hip_fail(c, e, "schedule launch");
  phase_mark(c, 1);
  nb::ForceArgs red{};
  rc = devcount_forces(c, pos_p, vel_p, mass, N, active, c->nact32, N, eps2, acc1, jerk1, pot1, false, &red);
  if (rc) return rc;
  phase_mark(c, 2);
  // the partial sums' reduce and the corrector in one pass
  const nb::StepArgs st{pos_p, vel_p, pos, vel, acc, jerk, t_tick, dt_level, eta, dt_max, max_level,
                        reinterpret_cast<unsigned long long*>(sched + 3),
                        reinterpret_cast<unsigned long long*>(sched + 2)};
  e = nb::launch_reduce_correct(c->prec, red, st, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "reduce and correct launch");
  phase_mark(c, 3);
  return NB_OK;
}


// Batched forces: the work list (system, i-block, j-chunk) is built on the
// host, largest items first, staged through pinned memory and walked by one
// launch (one workgroup per item; the hardware hands them out in list
// order, so the large items go first).  Each system's j-range is cut into
// chunks of about the same length J, chosen so the whole batch yields the
// item count below.
int nbody_forces_batch(nb_ctx* c, const int64_t* offsets, int64_t C, const double* eps2, const double* pos,
                       const double* vel, const double* mass, const int32_t* active, const int64_t* act_offsets,
                       double* acc, double* jerk, double* pot) {
  if (!c) return NB_EINVAL;
  if (C < 1 || C > (1 << 24) || !offsets || !eps2 || !act_offsets)
    return fail(c, NB_EINVAL, "C >= 1 and host offsets/eps2/act_offsets required%s");
  if (offsets[0] != 0 || act_offsets[0] != 0) return fail(c, NB_EINVAL, "offsets must start at 0%s");
  int64_t n_total = offsets[C], a_total = act_offsets[C];
  if (n_total < 1 || n_total >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "total rows must be in [1, 2^31)%s");
  bool any_mask = false;
  int64_t max_act = 0;
  for (int64_t s = 0; s < C; ++s) {
    if (offsets[s + 1] < offsets[s] || act_offsets[s + 1] < act_offsets[s])
      return fail(c, NB_EINVAL, "offsets and act_offsets must be non-decreasing%s");
    if (!finite_nonneg(eps2[s])) return fail(c, NB_EINVAL, "every eps2 must be finite and >= 0%s");
    if (act_offsets[s + 1] > act_offsets[s] && offsets[s + 1] == offsets[s])
      return fail(c, NB_EINVAL, "a system with active rows has no particles%s");
    any_mask = any_mask || kernel_mask(c->prec, eps2[s]);
    const int64_t na = act_offsets[s + 1] - act_offsets[s];
    if (na > max_act) max_act = na;
  }
  if (a_total == 0) return NB_OK;
  if (!pos || !vel || !mass || !active || !acc || !jerk || !pot) return fail(c, NB_EINVAL, "null pointer argument%s");
  // One kernel shape for the batch, from the mean active rows per system.
  Launch cfg = choose_batch(c, 1, (a_total + C - 1) / C, n_total, (a_total + C - 1) / C);
  if (any_mask) cfg.K = 1;  // an unsoftened system: the masked kernels hold one i-particle per lane
  if (cfg.L == 0) cfg.WG = nb::kBatchSjWG;
  log_launch(c, "batch forces", cfg, n_total, a_total);
  const int IB = nb::ib_of(cfg);
  // total work in (i-slot x j) units and the chunk length that splits it
  double work = 0.0;
  for (int64_t s = 0; s < C; ++s) {
    const int64_t na = act_offsets[s + 1] - act_offsets[s];
    work += (double)((na + IB - 1) / IB) * IB * (double)(offsets[s + 1] - offsets[s]);
  }
  // items wanted: three per resident workgroup on the scalar j-path (its
  // items start cheaply; 1.5-3 per slot measured best), eight per CU in the
  // LDS layout, whose items also stage tiles (more, shorter items measured
  // slower there)
  const double n_target = cfg.L == 0 ? 3.0 * c->num_cus * nb::batch_resident_wgs(c->prec, cfg, any_mask)
                                     : 8.0 * c->num_cus;
  double jt = work / ((double)IB * n_target);
  int64_t J = (int64_t)std::ceil(jt / nb::kTile) * nb::kTile;
  if (J < nb::kTile) J = nb::kTile;
  std::vector<nb::BatchSys> sys((size_t)C);
  std::vector<int32_t> nch((size_t)C);
  std::vector<nb::BatchItem> items;
  int64_t part_rows = 0;
  for (int64_t s = 0; s < C; ++s) {
    const int64_t nj = offsets[s + 1] - offsets[s];
    const int64_t na = act_offsets[s + 1] - act_offsets[s];
    int64_t S = (nj + J - 1) / J;
    const int64_t max_s = (nj + nb::kTile - 1) / nb::kTile;
    if (S > max_s) S = max_s;
    if (S < 1) S = 1;
    nch[s] = (int32_t)S;
    sys[s] = nb::BatchSys{offsets[s], offsets[s + 1], act_offsets[s], act_offsets[s + 1], eps2[s],
                          S > 1 ? part_rows : 0};
    if (S > 1) part_rows += S * na;
    const int64_t nib = (na + IB - 1) / IB;
    for (int64_t ch = 0; ch < S; ++ch)
      for (int64_t b = 0; b < nib; ++b) items.push_back(nb::BatchItem{(int32_t)s, (int32_t)b, (int32_t)ch, (int32_t)S});
  }
  // largest items first (cost ~ chunk length)
  std::stable_sort(items.begin(), items.end(), [&](const nb::BatchItem& x, const nb::BatchItem& y) {
    const int64_t lx = (sys[x.sys].j1 - sys[x.sys].j0 + x.nchunk - 1) / x.nchunk;
    const int64_t ly = (sys[y.sys].j1 - sys[y.sys].j0 + y.nchunk - 1) / y.nchunk;
    return lx > ly;
  });
  if (items.size() > (size_t)INT32_MAX) return fail(c, NB_EINVAL, "work list too long%s");
  const size_t b_items = items.size() * sizeof(nb::BatchItem);
  const size_t b_sys = sys.size() * sizeof(nb::BatchSys);
  const size_t b_nch = nch.size() * sizeof(int32_t);
  const size_t off_sys = (b_items + 255) / 256 * 256;
  const size_t off_nch = off_sys + (b_sys + 255) / 256 * 256;
  const size_t total = off_nch + b_nch;
  if (capturing(c->stream)) return fail(c, NB_ENOTSUP, "nbody_forces_batch stages its work list with a copy; it cannot be captured%s");
  if (total > c->batch_cap) {
    (void)hipStreamSynchronize(c->stream);
    if (c->batch_buf) (void)hipFree(c->batch_buf);
    c->batch_buf = nullptr;
    c->batch_cap = 0;
    if (hipMalloc(&c->batch_buf, total) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, NB_ENOMEM, "hipMalloc of the batch work list failed%s");
    }
    c->batch_cap = total;
  }
  if (!c->batch_ev && hipEventCreateWithFlags(&c->batch_ev, hipEventDisableTiming) != hipSuccess)
    return hip_fail(c, hipGetLastError(), "hipEventCreate");
  if (hipEventSynchronize(c->batch_ev) != hipSuccess) return hip_fail(c, hipGetLastError(), "batch staging wait");
  if (total > c->batch_host_cap) {
    if (c->batch_host) (void)hipHostFree(c->batch_host);
    c->batch_host = nullptr;
    c->batch_host_cap = 0;
    if (hipHostMalloc(&c->batch_host, total, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, NB_ENOMEM, "hipHostMalloc of the batch staging buffer failed%s");
    }
    c->batch_host_cap = total;
  }
  char* hb = static_cast<char*>(c->batch_host);
  std::memcpy(hb, items.data(), b_items);
  std::memcpy(hb + off_sys, sys.data(), b_sys);
  std::memcpy(hb + off_nch, nch.data(), b_nch);
  hipError_t e = hipMemcpyAsync(c->batch_buf, hb, total, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "batch work list copy");
  e = hipEventRecord(c->batch_ev, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "batch event");
  int rc = ensure_ws(c, (size_t)(part_rows > 0 ? part_rows : 1) * 7 * sizeof(double));
  if (rc) return rc;
  if (cfg.L == 0) {
    rc = ensure_mirror(c, n_total);
    if (rc) return rc;
  }
  char* db = static_cast<char*>(c->batch_buf);
  const nb::BatchItem* d_items = reinterpret_cast<const nb::BatchItem*>(db);
  const nb::BatchSys* d_sys = reinterpret_cast<const nb::BatchSys*>(db + off_sys);
  const int32_t* d_nch = reinterpret_cast<const int32_t*>(db + off_nch);
  e = nb::launch_batch(c->prec, cfg, d_items, (int)items.size(), nullptr, d_sys, pos, vel, mass, active, acc, jerk,
                       pot, static_cast<double*>(c->ws), part_rows, any_mask, 0, c->wq + nb::kErrorWord, c->mirror,
                       n_total, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "batch force launch");
  if (part_rows > 0) {
    e = nb::launch_batch_reduce(c->prec, d_sys, (int)C, d_nch, mass, active, a_total, acc, jerk, pot,
                                static_cast<double*>(c->ws), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "batch reduce launch");
  }
  return NB_OK;
}

// Block step over a batch of independent systems, planned on the device.
// The system table (offsets, softenings) is uploaded on the first call and
// whenever it changes (never during a capture); after that a step makes no
// host-device transfer and can be replayed from a graph.
extern "C" int nb_block_step_batch(nb_ctx* c, const int64_t* offsets, int64_t C, const double* eps2, double eta, double dt_max,
                        int32_t max_level, const double* mass, double* pos, double* vel, double* acc, double* jerk,
                        int64_t* t_tick, int32_t* dt_level, double* pos_p, double* vel_p, int32_t* active,
                        double* acc1, double* jerk1, double* pot1, int64_t* sched, int64_t t_stop_tick) {
  if (!c) return NB_EINVAL;
  if (C < 1 || C > (1 << 20) || !offsets || !eps2) return fail(c, NB_EINVAL, "C in [1, 2^20] and host offsets/eps2 required%s");
  if (offsets[0] != 0) return fail(c, NB_EINVAL, "offsets must start at 0%s");
  const int64_t N = offsets[C];
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "total rows must be in [1, 2^31)%s");
  bool any_mask = false;
  for (int64_t s = 0; s < C; ++s) {
    if (offsets[s + 1] < offsets[s]) return fail(c, NB_EINVAL, "offsets must be non-decreasing%s");
    if (!finite_nonneg(eps2[s])) return fail(c, NB_EINVAL, "every eps2 must be finite and >= 0%s");
    any_mask = any_mask || kernel_mask(c->prec, eps2[s]);
  }
  int rc = check_levels(c, eta, dt_max, max_level);
  if (rc) return rc;
  if (!mass || !pos || !vel || !acc || !jerk || !t_tick || !dt_level || !pos_p || !vel_p || !active || !acc1 ||
      !jerk1 || !pot1 || !sched)
    return fail(c, NB_EINVAL, "null pointer%s");
  rc = ensure_sched(c, N);
  if (rc) return rc;
  // one kernel shape for the batch, from the mean system size
  Launch cfg = choose_batch(c, 2, (N + C - 1) / C, N, (N + C - 1) / C);
  if (any_mask) cfg.K = 1;  // as in nbody_forces_batch
  if (cfg.L == 0) cfg.WG = nb::kBatchSjWG;
  log_launch(c, "batch block step", cfg, N, N);
  const int IB = nb::ib_of(cfg);
  // the scalar j-path runs its own workgroup size, which the single-system
  // occupancy table does not hold
  const int rgrid = cfg.L == 0 ? c->num_cus * nb::batch_resident_wgs(c->prec, cfg, any_mask)
                               : resident_grid(c, cfg, any_mask);
  const int target = 2 * rgrid;
  const int max_items = target + (int)((N + IB - 1) / IB) + (int)C + 64;
  const int64_t part_cap = (int64_t)IB * target + N;
  // device system table and work list
  const size_t o_off = 0;
  const size_t o_eps = o_off + ((size_t)(C + 1) * 8 + 255) / 256 * 256;
  const size_t o_sys = o_eps + ((size_t)C * 8 + 255) / 256 * 256;
  const size_t o_nch = o_sys + ((size_t)C * sizeof(nb::BatchSys) + 255) / 256 * 256;
  const size_t o_items = o_nch + ((size_t)C * 4 + 255) / 256 * 256;
  const size_t o_nit = o_items + ((size_t)max_items * sizeof(nb::BatchItem) + 255) / 256 * 256;
  const size_t total = o_nit + 256;
  const bool same = c->bp_buf && c->bp_off.size() == (size_t)C + 1 &&
                    std::equal(c->bp_off.begin(), c->bp_off.end(), offsets) &&
                    std::equal(c->bp_eps2.begin(), c->bp_eps2.end(), eps2) && total <= c->bp_cap;
  if (!same) {
    if (capturing(c->stream)) return fail(c, NB_ENOTSUP, "the batch table changed during a capture; run one step first%s");
    (void)hipStreamSynchronize(c->stream);
    if (total > c->bp_cap) {
      if (c->bp_buf) (void)hipFree(c->bp_buf);
      c->bp_buf = nullptr;
      c->bp_cap = 0;
      if (hipMalloc(&c->bp_buf, total) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, NB_ENOMEM, "hipMalloc of the batch plan failed%s");
      }
      c->bp_cap = total;
    }
    char* b = static_cast<char*>(c->bp_buf);
    if (hipMemcpy(b + o_off, offsets, (size_t)(C + 1) * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b + o_eps, eps2, (size_t)C * 8, hipMemcpyHostToDevice) != hipSuccess)
      return hip_fail(c, hipGetLastError(), "batch table upload");
    c->bp_off.assign(offsets, offsets + C + 1);
    c->bp_eps2.assign(eps2, eps2 + C);
  }
  rc = ensure_ws(c, (size_t)part_cap * 7 * sizeof(double));
  if (rc) return rc;
  if (cfg.L == 0) {
    rc = ensure_mirror(c, N);
    if (rc) return rc;
  }
  char* b = static_cast<char*>(c->bp_buf);
  const int64_t* d_off = reinterpret_cast<const int64_t*>(b + o_off);
  const double* d_eps = reinterpret_cast<const double*>(b + o_eps);
  nb::BatchSys* d_sys = reinterpret_cast<nb::BatchSys*>(b + o_sys);
  int32_t* d_nch = reinterpret_cast<int32_t*>(b + o_nch);
  nb::BatchItem* d_items = reinterpret_cast<nb::BatchItem*>(b + o_items);
  int* d_nit = reinterpret_cast<int*>(b + o_nit);
  const double dt_min = std::ldexp(dt_max, -max_level);
  const nb::PredictArgs pred{pos, vel, acc, jerk, dt_min, pos_p, vel_p};
  phase_mark(c, 0);
  hipError_t e = nb::launch_schedule(t_tick, dt_level, N, max_level, active, sched, c->sched_tmp, c->sched_cnt,
                                     c->nact32, t_stop_tick, c->stop_dev, c->stream, &pred);
  if (e != hipSuccess) return hip_fail(c, e, "schedule launch");
  e = nb::launch_batch_plan(d_off, d_eps, (int)C, active, sched + 1, IB, target, d_sys, d_nch, d_items, max_items,
                            d_nit, part_cap, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "batch plan launch");
  phase_mark(c, 1);
  e = nb::launch_batch(c->prec, cfg, d_items, max_items, d_nit, d_sys, pos_p, vel_p, mass, active, acc1, jerk1, pot1,
                       static_cast<double*>(c->ws), part_cap, any_mask, rgrid, c->wq + nb::kErrorWord, c->mirror, N,
                       c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "batch force launch");
  phase_mark(c, 2);
  const nb::StepArgs sa{pos_p, vel_p, pos, vel, acc, jerk, t_tick, dt_level, eta, dt_max, max_level,
                        reinterpret_cast<unsigned long long*>(sched + 3),
                        reinterpret_cast<unsigned long long*>(sched + 2)};
  e = nb::launch_batch_reduce_correct(c->prec, d_sys, d_nch, (int)C, sched + 1, N, mass, active, acc1, jerk1, pot1,
                                      static_cast<double*>(c->ws), sa, c->wq + nb::kErrorWord, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "batch reduce-correct launch");
  phase_mark(c, 3);
  return NB_OK;
}

int nb_energy(nb_ctx* c, const double* pos, const double* vel, const double* mass, const double* pot, int64_t N,
              double* out) {
  if (!c) return NB_EINVAL;
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(c, NB_EINVAL, "N must be in [1, 2^31)%s");
  if (!pos || !vel || !mass || !pot || !out) return fail(c, NB_EINVAL, "null pointer%s");
  int rc = ensure_energy(c, N);
  if (rc) return rc;
  hipError_t e = nb::launch_energy(pos, vel, mass, pot, N, c->energy_part, out, c->stream);
  return e == hipSuccess ? NB_OK : hip_fail(c, e, "energy launch");
}

}  // extern "C"
