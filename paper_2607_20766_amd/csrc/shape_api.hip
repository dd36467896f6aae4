// C-ABI layer of the IS shape-overlap engine: argument validation, context
// scratch, launches.  No exception crosses the ABI.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "shape_is.h"
#include "shape_kernels.hpp"

#define SHAPE_VERSION_STR "shape_is 0.1.0 (gfx950)"

namespace {

struct Buffer {
  void* ptr = nullptr;
  size_t bytes = 0;
};

enum Slot {
  S_Q_ATOM, S_Q_SAMP, S_Q_Z, S_Q_ID, S_Q_BAD, S_Q_CENTRE,
  S_L_ATOM, S_L_SAMP, S_L_Z, S_L_ID, S_L_BAD, S_L_CENTRE,
  S_PARTIALS, S_RESULT, S_QS, S_QF2,
  S_SELF_A, S_SELF_B,
  S_MSE, S_TOPK_SEL, S_TOPK_HIST, S_TOPK_GT, S_TOPK_EQ, S_COLSUM, S_TUNE, S_MLP_PACK, S_FEAT_MOM, S_GEMM_PART,
  S_GRID_BOX, S_GRID_TAB, S_GRID_PART, S_PEAK, S_MLP_D, S_MLP_STEP, S_ORDER,
  S_COUNT
};

}  // namespace

// Identity of the molecule set last prepared into one family of slots.
struct PrepKey {
  bool valid = false;
  const void *off = nullptr, *xyz = nullptr, *alpha = nullptr, *id = nullptr;
  int64_t n_atoms = 0;
  int32_t n_mols = 0, max_atoms = 0;
  shape::Prepared P{};
  bool same(const shape_mols* m) const {
    return valid && off == m->atom_offset && xyz == m->xyz && alpha == m->alpha &&
           id == m->mol_id && n_atoms == m->n_atoms && n_mols == m->n_mols &&
           max_atoms == m->max_atoms;
  }
};

// Executable graphs replay the device addresses they captured.  A scratch
// buffer that grows while any graph of its context is alive is therefore not
// freed but retired, and retired buffers are released once the last of those
// graphs is destroyed (or with the context).  Shared by the context and its
// graphs, so a graph may outlive its context.
struct GraphLife {
  std::mutex m;
  int device = -1;
  int live = 0;                 // graphs instantiated and not yet destroyed
  std::vector<void*> retired;   // buffers replaced while graphs were alive
  size_t retired_bytes = 0;
};

struct shape_ctx {
  int device = -1;
  std::shared_ptr<GraphLife> life;
  int n_cu = 0;
  char arch[64] = {0};          // gcnArchName of the device
  int fail_allocs = 0;          // scratch allocations still to refuse (failure injection)
  size_t lds_per_block = 0;
  std::string err;
  Buffer buf[S_COUNT];
  int* flag = nullptr;  // device int[3]: invalid-data flag, then one per slot family
  bool prep_cache = false;  // reuse the last preparation of an unchanged set
  PrepKey prepared[2];      // query-side and library-side slot families
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  int screen_variant = -1;        // -1: default tile shape
  int sampling = SHAPE_SAMPLING_IID;
  bool capturing = false;         // a graph capture is open on capture_stream
  bool capture_failed = false;    // a call failed while capturing
  hipStream_t capture_stream = nullptr;
  void* noalloc = nullptr;        // device address of this GPU's copy of `scratch`
};

struct shape_graph {
  hipGraphExec_t exec = nullptr;
  int device = -1;
  std::shared_ptr<GraphLife> life;  // the capturing context's graph bookkeeping
};

// ---------------------------------------------------------------------------
// Fixed scratch of shape_estimate_noalloc: a file-scope device array, one copy
// per GPU (each GPU's copy has its own address, looked up once per context at
// creation), held until the process ends.  Host code never passes the array's
// name to a kernel: in host code it is only a stand-in symbol.  Layout: the
// prepared records of the two one-molecule sets (at most SHAPE_MAX_ATOMS atoms
// each), the per-block partial sums of est_blocks(SHAPE_NOALLOC_MAX_SAMPLES)
// blocks per side, and the device copy of the result.
// ---------------------------------------------------------------------------
namespace {

struct NoallocLayout {
  size_t atom[2], samp[2], Z, id, bad, centre, partials, result, total;
  int max_blocks;
  NoallocLayout() {
    size_t o = 0;
    auto take = [&o](size_t bytes) {
      const size_t at = o;
      o += (bytes + 255) & ~(size_t)255;
      return at;
    };
    for (int s = 0; s < 2; ++s) {
      atom[s] = take(SHAPE_MAX_ATOMS * sizeof(shape::Atom));
      samp[s] = take(SHAPE_MAX_ATOMS * sizeof(shape::AtomSampling));
    }
    Z = take(2 * sizeof(double));
    id = take(2 * sizeof(uint32_t));
    bad = take(2 * sizeof(int));
    centre = take(2 * sizeof(float4));
    max_blocks = shape::est_blocks(SHAPE_NOALLOC_MAX_SAMPLES);
    partials = take((size_t)2 * max_blocks * shape::kEstSums * sizeof(double));
    result = take(sizeof(shape_result));
    total = o;
  }
};

// 2 x 8192 blocks x 11 doubles of partials dominate: 1.39 MiB in all
constexpr size_t kNoallocScratchBytes = (size_t)3 << 19;  // 1.5 MiB

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

thread_local std::string g_create_err;

int fail(shape_ctx* c, int code, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  if (c) {
    c->err = msg;
    if (c->capturing) c->capture_failed = true;
  } else {
    g_create_err = msg;
  }
  return code;
}

int hip_fail(shape_ctx* c, hipError_t e, const char* what) {
  return fail(c, SHAPE_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr, what)                     \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
  } while (0)

// Grow-only scratch.  Freed buffers are released after a device sync so a
// buffer still in use by queued work is never returned to the allocator.
int ensure(shape_ctx* c, Slot s, size_t bytes, void** out) {
  Buffer& b = c->buf[s];
  if (b.bytes < bytes) {
    if (c->capturing)
      return fail(c, SHAPE_E_UNSUPPORTED,
                  "scratch would grow during graph capture: make the same calls once "
                  "before capturing");
    if (c->fail_allocs > 0) {  // injected failure: the slot keeps its old buffer
      --c->fail_allocs;
      return fail(c, SHAPE_E_NOMEM, "scratch allocation of %zu bytes refused (injected)",
                  bytes);
    }
    if (b.ptr) {
      std::lock_guard<std::mutex> lk(c->life->m);
      if (c->life->live > 0) {
        // a live graph may still replay with this address
        c->life->retired.push_back(b.ptr);
        c->life->retired_bytes += b.bytes;
      } else {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
        (void)hipFree(b.ptr);
      }
      b.ptr = nullptr;
      b.bytes = 0;
    }
    size_t want = bytes + bytes / 4 + 256;
    hipError_t e = hipMalloc(&b.ptr, want);
    if (e != hipSuccess) {
      b.ptr = nullptr;
      return fail(c, SHAPE_E_NOMEM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    }
    b.bytes = want;
  }
  *out = b.ptr;
  return SHAPE_OK;
}

int set_device(shape_ctx* c) {
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  return SHAPE_OK;
}

int check_mols(shape_ctx* c, const shape_mols* m, const char* name, bool single) {
  if (!m) return fail(c, SHAPE_E_INVAL, "%s is NULL", name);
  if (m->n_mols < 1) return fail(c, SHAPE_E_RANGE, "%s->n_mols = %d < 1", name, m->n_mols);
  if (single && m->n_mols != 1)
    return fail(c, SHAPE_E_RANGE, "%s must hold exactly one molecule (n_mols = %d)", name,
                m->n_mols);
  if (m->max_atoms < 1 || m->max_atoms > SHAPE_MAX_ATOMS)
    return fail(c, SHAPE_E_RANGE, "%s->max_atoms = %d outside [1, %d]", name, m->max_atoms,
                SHAPE_MAX_ATOMS);
  if (m->n_atoms < 1 || m->n_atoms > (int64_t)0x7FFFFFFF)
    return fail(c, SHAPE_E_RANGE, "%s->n_atoms = %lld outside [1, 2^31)", name,
                (long long)m->n_atoms);
  if (!m->atom_offset || !m->xyz || !m->alpha)
    return fail(c, SHAPE_E_INVAL, "%s has a NULL array", name);
  return SHAPE_OK;
}

// Prepare a molecule set into the query (q = true) or library slots.
// subset (device int32 [n_subset], optional): prepare only these molecules
// (records at their usual places; the rest of the slots stay as they were),
// for calls that read no other molecule.  Such a partial preparation is
// never kept for reuse.
int prepare(shape_ctx* c, const shape_mols* m, bool q, hipStream_t st, shape::Prepared* P,
            const int32_t* subset = nullptr, int32_t n_subset = 0) {
  const int base = q ? S_Q_ATOM : S_L_ATOM;
  PrepKey& key = c->prepared[q ? 0 : 1];
  int* set_flag = c->flag + (q ? 1 : 2);
  if (c->prep_cache && key.same(m)) {
    *P = key.P;
    HIP_TRY(c, shape::launch_flag_or(c->flag, set_flag, st), "flag kernel");
    return SHAPE_OK;
  }
  key.valid = false;
  void* p[6];
  int rc;
  const size_t na = (size_t)m->n_atoms, nm = (size_t)m->n_mols;
  if ((rc = ensure(c, (Slot)(base + 0), na * sizeof(shape::Atom), &p[0]))) return rc;
  if ((rc = ensure(c, (Slot)(base + 1), na * sizeof(shape::AtomSampling), &p[1]))) return rc;
  if ((rc = ensure(c, (Slot)(base + 2), nm * sizeof(double), &p[2]))) return rc;
  if ((rc = ensure(c, (Slot)(base + 3), nm * sizeof(uint32_t), &p[3]))) return rc;
  if ((rc = ensure(c, (Slot)(base + 4), nm * sizeof(int), &p[4]))) return rc;
  if ((rc = ensure(c, (Slot)(base + 5), nm * sizeof(float4), &p[5]))) return rc;
  P->atom = (shape::Atom*)p[0];
  P->samp = (shape::AtomSampling*)p[1];
  P->Z = (double*)p[2];
  P->id = (uint32_t*)p[3];
  P->bad = (int*)p[4];
  P->centre = (float4*)p[5];
  shape::MolsDev in{m->n_mols, m->max_atoms, m->n_atoms, m->atom_offset, m->xyz, m->alpha,
                    m->mol_id};
  if (subset) {
    HIP_TRY(c, shape::launch_prepare(in, *P, c->flag, nullptr, st, subset, n_subset),
            "prepare kernel");
    return SHAPE_OK;
  }
  if (c->prep_cache) HIP_TRY(c, shape::launch_fill_int(set_flag, 1, 0, st), "flag reset");
  HIP_TRY(c, shape::launch_prepare(in, *P, c->flag, c->prep_cache ? set_flag : nullptr, st),
          "prepare kernel");
  if (c->prep_cache) {
    key.off = m->atom_offset;
    key.xyz = m->xyz;
    key.alpha = m->alpha;
    key.id = m->mol_id;
    key.n_atoms = m->n_atoms;
    key.n_mols = m->n_mols;
    key.max_atoms = m->max_atoms;
    key.P = *P;
    key.valid = true;
  }
  return SHAPE_OK;
}

// Calls that synchronise cannot be recorded into a graph.
int refuse_in_capture(shape_ctx* c, const char* what) {
  return fail(c, SHAPE_E_UNSUPPORTED, "%s synchronises and cannot run during graph capture",
              what);
}

uint2 key_of(uint64_t seed) { return make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)); }

// Brackets the dominant kernel of a call with HIP events when timing is on.
struct KernelTimer {
  shape_ctx* c;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  KernelTimer(shape_ctx* c_, hipStream_t st_) : c(c_), st(st_) {
    if (!c->timing || c->capturing) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess ||
        hipEventRecord(a, st) != hipSuccess) {
      a = b = nullptr;
    }
  }
  void stop() {
    if (!a) return;
    if (hipEventRecord(b, st) == hipSuccess) c->events.emplace_back(a, b);
    a = b = nullptr;
  }
};

// A named roctx range around one entry point's host work and launches (a
// no-op unless a profiler listens), so traces attribute kernels to calls.
struct ProfRange {
  explicit ProfRange(const char* name) { roctxRangePushA(name); }
  ~ProfRange() { roctxRangePop(); }
  ProfRange(const ProfRange&) = delete;
  ProfRange& operator=(const ProfRange&) = delete;
};

// Grids of one workgroup per pair are launched in the order
// shape::launch_work_order computes (largest estimated work first; a few
// microseconds) when they hold at least this many pairs per compute unit:
// fewer run in a few waves of workgroups, where the order hardly changes
// when the last ones finish.  Screens run up to eight 64-lane workgroups per
// SIMD, alignments four 256-lane workgroups per compute unit.
constexpr int kOrderScreenPerCu = 16;
constexpr int kOrderAlignPerCu = 4;
constexpr int kOrderFoAlignPerCu = 16;
// Features: the order groups molecules of one size into a wave (it matters
// at any size, but its three launches cost a few microseconds).
constexpr int kOrderFeaturesPerCu = 512;

// The context's launch-order buffers for n pairs (the sort's work area, then
// the order), or nullptr when the grid is too short for the order to matter.
struct WorkOrder {
  int* work = nullptr;
  int* order = nullptr;
};
int work_order_slot(shape_ctx* c, int64_t n, int min_per_cu, WorkOrder* w) {
  *w = WorkOrder{};
  if (n < (int64_t)min_per_cu * c->n_cu) return SHAPE_OK;
  void* buf;
  const size_t ints = (size_t)shape::work_order_ints() + (size_t)n;
  const int rc = ensure(c, S_ORDER, ints * sizeof(int), &buf);  // hipMalloc: aligned
  if (rc) return rc;
  w->work = (int*)buf;
  w->order = w->work + shape::work_order_ints();
  return SHAPE_OK;
}

// Work of an alignment pair in atoms' worth, per CRN sample: A's atoms and
// sampling once, then per start and step the forward and adjoint passes over
// B's atoms (about two evaluations per atom) and the per-sample weight and
// gradient steps.
shape::OrderArgs align_order_args(const shape_mols* A, const shape_mols* B, int n_starts,
                                  int n_steps) {
  const uint32_t S = (uint32_t)std::min<int64_t>((int64_t)(n_steps + 1) * n_starts, 1 << 20);
  shape::OrderArgs o{};
  o.n = A->n_mols;
  o.per_xcd = 0;
  o.offA = A->atom_offset;
  o.nA_mols = A->n_mols;
  o.max_a = A->max_atoms;
  o.offB = B->atom_offset;
  o.nB_mols = B->n_mols;
  o.max_b = B->max_atoms;
  o.wA = 1;
  o.wB = 2 * S;
  o.w0 = 24 + 4 * S;
  return o;
}

// Validation, molecule preparation and the query-side sample cache of a
// screen; fills the kernel arguments (a->n_pairs = 0: nothing to launch).
int screen_setup(shape_ctx* c, const shape_mols* query, const shape_mols* lib,
                 const int32_t* pairs, int32_t n_pairs, const shape_screen_params* prm,
                 hipStream_t st, const shape_screen_out* out, shape::ScreenArgs* a) {
  int rc;
  if ((rc = check_mols(c, query, "query", true))) return rc;
  if ((rc = check_mols(c, lib, "lib", false))) return rc;
  if (!prm || !out) return fail(c, SHAPE_E_INVAL, "params or out is NULL");
  if (n_pairs < 0) return fail(c, SHAPE_E_RANGE, "n_pairs < 0");
  if (n_pairs > 0 && (!out->T || !out->se_T))
    return fail(c, SHAPE_E_INVAL, "out->T and out->se_T are required");
  if (!pairs && n_pairs > lib->n_mols)
    return fail(c, SHAPE_E_RANGE, "n_pairs = %d exceeds lib->n_mols = %d", n_pairs,
                lib->n_mols);
  int64_t n_fixed = 0, cap = 0;
  int round_side = 0;
  const bool anti = c->sampling == SHAPE_SAMPLING_ANTITHETIC;
  if (prm->mode == SHAPE_SCREEN_FIXED) {
    if (prm->n_per_side < 64 || prm->n_per_side > (1 << 20) || prm->n_per_side % 64)
      return fail(c, SHAPE_E_RANGE, "n_per_side must be a multiple of 64 in [64, 2^20]");
    if (anti && prm->n_per_side % 128)
      return fail(c, SHAPE_E_RANGE, "antithetic sampling needs n_per_side a multiple of 128");
    n_fixed = prm->n_per_side;
    round_side = (int)(n_fixed % 256 == 0 ? 256 : (anti ? 128 : 64));
  } else if (prm->mode == SHAPE_SCREEN_ADAPTIVE) {
    if (prm->round_per_pair < 128 || prm->round_per_pair > 8192 || prm->round_per_pair % 128)
      return fail(c, SHAPE_E_RANGE, "round_per_pair must be a multiple of 128 in [128, 8192]");
    if (anti && prm->round_per_pair % 256)
      return fail(c, SHAPE_E_RANGE, "antithetic sampling needs round_per_pair a multiple of 256");
    if (prm->cap_per_pair < prm->round_per_pair || prm->cap_per_pair > (1 << 21) ||
        prm->cap_per_pair % prm->round_per_pair)
      return fail(c, SHAPE_E_RANGE,
                  "cap_per_pair must be a multiple of round_per_pair, at most 2^21");
    if (!(prm->tau > 0.0) || !isfinite(prm->tau))
      return fail(c, SHAPE_E_RANGE, "tau must be finite and > 0");
    round_side = prm->round_per_pair / 2;
    cap = prm->cap_per_pair;
  } else {
    return fail(c, SHAPE_E_INVAL, "unknown mode %d", prm->mode);
  }
  if (n_pairs == 0) {
    a->n_pairs = 0;
    return SHAPE_OK;
  }
  if ((rc = set_device(c))) return rc;
  shape::Prepared PQ, PL;
  if ((rc = prepare(c, query, true, st, &PQ))) return rc;
  // a screen of a small subset of a large library prepares only that subset
  // (unless the whole set is already prepared for reuse)
  const bool subset = pairs && (int64_t)n_pairs * 4 < lib->n_mols &&
                      !(c->prep_cache && c->prepared[1].same(lib));
  if ((rc = prepare(c, lib, false, st, &PL, subset ? pairs : nullptr, subset ? n_pairs : 0)))
    return rc;
  const int64_t n_cache = prm->mode == SHAPE_SCREEN_FIXED ? n_fixed : cap / 2;
  void *qs, *qf2;
  if ((rc = ensure(c, S_QS, (size_t)n_cache * sizeof(float4), &qs))) return rc;
  if ((rc = ensure(c, S_QF2, (size_t)n_cache * sizeof(float), &qf2))) return rc;
  // a screen of many pairs runs them longest first (results do not depend on
  // the order; the last workgroups then finish closer together)
  WorkOrder wo;
  if ((rc = work_order_slot(c, n_pairs, kOrderScreenPerCu, &wo))) return rc;
  const uint2 key = key_of(prm->seed);
  HIP_TRY(c, shape::launch_query_cache(PQ, query->atom_offset, n_cache, key, anti ? 1 : 0,
                                       (float4*)qs,
                                       (float*)qf2, st),
          "query cache kernel");
  a->Q = PQ;
  a->offQ = query->atom_offset;
  a->max_q = query->max_atoms;
  a->L = PL;
  a->offL = lib->atom_offset;
  a->n_lib = lib->n_mols;
  a->max_b = lib->max_atoms;
  a->qs = (const float4*)qs;
  a->qf2 = (const float*)qf2;
  a->pairs = pairs;
  a->n_pairs = n_pairs;
  a->mode = prm->mode;
  a->n_fixed = n_fixed;
  a->round_side = round_side;
  a->cap_pair = cap;
  a->tau = prm->tau;
  a->key = key;
  a->n_start = prm->mode == SHAPE_SCREEN_ADAPTIVE ? prm->n_start : nullptr;
  a->anti = anti ? 1 : 0;
  a->T = out->T;
  a->se_T = out->se_T;
  a->O_ab = out->O_ab;
  a->O_aa = out->O_aa;
  a->O_bb = out->O_bb;
  a->n_used = out->n_used;
  a->order = nullptr;
  if (wo.order) {
    // per pair of samples: N_B evaluations at the query's sample, N_B + N_A
    // at the library's, and Philox, inverse normals, component choice and
    // weights, worth about 24 evaluations; times the rounds of a seeded budget
    shape::OrderArgs o{};
    o.n = n_pairs;
    o.per_xcd = 1;
    o.pairs = pairs;
    o.offA = query->atom_offset;
    o.nA_mols = 1;
    o.max_a = query->max_atoms;
    o.a_single = 1;
    o.offB = lib->atom_offset;
    o.nB_mols = lib->n_mols;
    o.max_b = lib->max_atoms;
    o.wA = 1;
    o.wB = 2;
    o.w0 = 24;
    o.n_start = a->n_start;
    o.round_pair = 2 * (int64_t)round_side;
    o.cap = cap;
    HIP_TRY(c, shape::launch_work_order(o, wo.order, wo.work, st), "launch order kernels");
    a->order = wo.order;
  }
  return SHAPE_OK;
}

int screen_variant_of(const shape_ctx* c) { return c->screen_variant < 0 ? 0 : c->screen_variant; }

}  // namespace

extern "C" {


const char* shape_version(void) { return SHAPE_VERSION_STR; }

int shape_create(shape_ctx** out, int device) {
  if (!out) return fail(nullptr, SHAPE_E_INVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0)
    return fail(nullptr, SHAPE_E_HIP, "no HIP device available (%s)",
                e != hipSuccess ? hipGetErrorString(e) : "count 0");
  if (device < 0 || device >= n)
    return fail(nullptr, SHAPE_E_RANGE, "device %d outside [0, %d)", device, n);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return fail(nullptr, SHAPE_E_HIP, "hipGetDeviceProperties: %s",
                                   hipGetErrorString(e));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, SHAPE_E_UNSUPPORTED, "device %d is %s, not gfx950", device,
                prop.gcnArchName);
  shape_ctx* c = new (std::nothrow) shape_ctx();
  if (!c) return fail(nullptr, SHAPE_E_NOMEM, "context allocation failed");
  try {
    c->life = std::make_shared<GraphLife>();
  } catch (...) {
    delete c;
    return fail(nullptr, SHAPE_E_NOMEM, "context allocation failed");
  }
  c->life->device = device;
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
  c->lds_per_block = prop.sharedMemPerBlock;
  e = hipSetDevice(device);
  if (e == hipSuccess) e = hipMalloc(&c->flag, 3 * sizeof(int));
  if (e == hipSuccess) e = hipMemset(c->flag, 0, 3 * sizeof(int));
  // this device's copy of the allocation-free entry point's scratch (the
  // device is current here; every GPU holds the array at its own address)
  if (e == hipSuccess) e = hipGetSymbolAddress(&c->noalloc, HIP_SYMBOL(scratch));
  if (e != hipSuccess) {
    if (c->flag) (void)hipFree(c->flag);
    delete c;
    return fail(nullptr, SHAPE_E_HIP, "context set-up: %s", hipGetErrorString(e));
  }
  *out = c;
  return SHAPE_OK;
}

void shape_destroy(shape_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (auto& b : c->buf)
    if (b.ptr) (void)hipFree(b.ptr);
  {
    // graphs that outlive the context can no longer be launched (a launch
    // needs the context), so nothing replays with these addresses again
    std::lock_guard<std::mutex> lk(c->life->m);
    for (void* p : c->life->retired) (void)hipFree(p);
    c->life->retired.clear();
    c->life->retired_bytes = 0;
  }
  for (auto& e : c->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (c->flag) (void)hipFree(c->flag);
  delete c;
}

const char* shape_last_error(const shape_ctx* c) {
  return c ? c->err.c_str() : g_create_err.c_str();
}

int shape_alpha_from_radius(shape_ctx* c, const float* radius, int64_t n, double lambda,
                            float* alpha, void* stream) {
  if (!c) return SHAPE_E_INVAL;
  try {
    if (n < 0) return fail(c, SHAPE_E_RANGE, "n = %lld < 0", (long long)n);
    if (n > 0 && (!radius || !alpha)) return fail(c, SHAPE_E_INVAL, "NULL array");
    if (!(lambda > 0.0) || !isfinite(lambda))
      return fail(c, SHAPE_E_INVAL, "lambda must be finite and > 0");
    int rc = set_device(c);
    if (rc) return rc;
    const double kappa = M_PI * pow(3.0 / (4.0 * M_PI), 2.0 / 3.0);
    HIP_TRY(c, shape::launch_alpha_from_radius(radius, n, kappa, lambda, alpha,
                                               (hipStream_t)stream),
            "alpha kernel");
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

}  // extern "C"

namespace {

// Argument checks shared by shape_estimate and shape_estimate_noalloc.
int estimate_check(shape_ctx* c, const shape_mols* A, const shape_mols* B, int64_t n_a,
                   int64_t n_b, const shape_result* out, int64_t max_n) {
  int rc;
  if ((rc = check_mols(c, A, "A", true))) return rc;
  if ((rc = check_mols(c, B, "B", true))) return rc;
  if (!out) return fail(c, SHAPE_E_INVAL, "out is NULL");
  if (n_a < 2 || n_b < 2 || n_a > max_n || n_b > max_n)
    return fail(c, SHAPE_E_RANGE, "sample counts must lie in [2, %lld]", (long long)max_n);
  const int anti = c->sampling == SHAPE_SAMPLING_ANTITHETIC ? 1 : 0;
  if (anti && (n_a % 2 || n_b % 2 || n_a < 4 || n_b < 4))
    return fail(c, SHAPE_E_RANGE, "antithetic sampling needs even sample counts >= 4");
  return SHAPE_OK;
}

}  // namespace

extern "C" {

int shape_estimate(shape_ctx* c, const shape_mols* A, const shape_mols* B, int64_t n_a,
                   int64_t n_b, uint64_t seed, void* stream, shape_result* out) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_estimate");
  if (c->capturing) return refuse_in_capture(c, "shape_estimate");
  try {
    int rc;
    if ((rc = estimate_check(c, A, B, n_a, n_b, out, (int64_t)1 << 31))) return rc;
    const int anti = c->sampling == SHAPE_SAMPLING_ANTITHETIC ? 1 : 0;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    shape::Prepared PA, PB;
    if ((rc = prepare(c, A, true, st, &PA))) return rc;
    if ((rc = prepare(c, B, false, st, &PB))) return rc;
    const int64_t units = (n_a > n_b ? n_a : n_b) / (anti ? 2 : 1);
    const int nblk = shape::est_blocks(units);
    void *partials, *res;
    if ((rc = ensure(c, S_PARTIALS, (size_t)2 * nblk * shape::kEstSums * sizeof(double),
                     &partials)))
      return rc;
    if ((rc = ensure(c, S_RESULT, sizeof(shape_result), &res))) return rc;
    // invalid inputs are reported before the sampling kernels read them
    int bad[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(&bad[0], PA.bad, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
    HIP_TRY(c, hipMemcpyAsync(&bad[1], PB.bad, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
    HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    if (bad[0] || bad[1]) {
      HIP_TRY(c, shape::launch_fill_int(c->flag, 1, 0, st), "flag reset");
      return fail(c, SHAPE_E_DATA, "invalid molecule data in %s", bad[0] ? "A" : "B");
    }
    KernelTimer timer(c, st);
    HIP_TRY(c, shape::launch_estimate(PA, PB, A->atom_offset, B->atom_offset, n_a, n_b,
                                      key_of(seed), anti, (double*)partials, nblk,
                                      (shape_result*)res, st),
            "estimate kernels");
    timer.stop();
    HIP_TRY(c, hipMemcpyAsync(out, res, sizeof(shape_result), hipMemcpyDeviceToHost, st),
            "result copy");
    HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_estimate_noalloc(shape_ctx* c, const shape_mols* A, const shape_mols* B,
                           int64_t n_a, int64_t n_b, uint64_t seed, void* stream,
                           shape_result* out) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_estimate_noalloc");
  if (c->capturing) return refuse_in_capture(c, "shape_estimate_noalloc");
  try {
    int rc;
    if ((rc = estimate_check(c, A, B, n_a, n_b, out, SHAPE_NOALLOC_MAX_SAMPLES))) return rc;
    // records are written at atom_offset[0] + i < n_atoms: the whole set must
    // fit the fixed per-side staging
    if (A->n_atoms > SHAPE_MAX_ATOMS || B->n_atoms > SHAPE_MAX_ATOMS)
      return fail(c, SHAPE_E_RANGE, "n_atoms of A and B must be at most %d here",
                  SHAPE_MAX_ATOMS);
    const NoallocLayout L;
    if (L.total > kNoallocScratchBytes || !c->noalloc)
      return fail(c, SHAPE_E_HIP, "fixed scratch unavailable");
    const int anti = c->sampling == SHAPE_SAMPLING_ANTITHETIC ? 1 : 0;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)c->noalloc;  // this GPU's copy, never the symbol's name
    shape::Prepared P[2];
    const shape_mols* M[2] = {A, B};
    for (int s = 0; s < 2; ++s) {
      P[s].atom = (shape::Atom*)(base + L.atom[s]);
      P[s].samp = (shape::AtomSampling*)(base + L.samp[s]);
      P[s].Z = (double*)(base + L.Z) + s;
      P[s].id = (uint32_t*)(base + L.id) + s;
      P[s].bad = (int*)(base + L.bad) + s;
      P[s].centre = (float4*)(base + L.centre) + s;
      const shape::MolsDev in{M[s]->n_mols,     M[s]->max_atoms, M[s]->n_atoms,
                              M[s]->atom_offset, M[s]->xyz,       M[s]->alpha,
                              M[s]->mol_id};
      // every record the kernels read below is written here (the one
      // molecule's Z, id, flag, centre and its atoms): nothing has to start
      // at zero
      HIP_TRY(c, shape::launch_prepare(in, P[s], c->flag, nullptr, st), "prepare kernel");
    }
    const int64_t units = (n_a > n_b ? n_a : n_b) / (anti ? 2 : 1);
    const int nblk = shape::est_blocks(units);  // <= L.max_blocks by the range check
    int bad[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(bad, base + L.bad, sizeof bad, hipMemcpyDeviceToHost, st),
            "copy");
    HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    if (bad[0] || bad[1]) {
      HIP_TRY(c, shape::launch_fill_int(c->flag, 1, 0, st), "flag reset");
      return fail(c, SHAPE_E_DATA, "invalid molecule data in %s", bad[0] ? "A" : "B");
    }
    shape_result* res = (shape_result*)(base + L.result);
    HIP_TRY(c, shape::launch_estimate(P[0], P[1], A->atom_offset, B->atom_offset, n_a, n_b,
                                      key_of(seed), anti, (double*)(base + L.partials), nblk,
                                      res, st),
            "estimate kernels");
    HIP_TRY(c, hipMemcpyAsync(out, res, sizeof(shape_result), hipMemcpyDeviceToHost, st),
            "result copy");
    HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_sample_points(shape_ctx* c, const shape_mols* M, int32_t mol, int64_t k0, int32_t n,
                        uint64_t seed, void* stream, uint32_t* thr, uint32_t* words,
                        int32_t* comp, float* r) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_sample_points");
  if (c->capturing) return refuse_in_capture(c, "shape_sample_points");
  try {
    int rc;
    if ((rc = check_mols(c, M, "M", false))) return rc;
    if (mol < 0 || mol >= M->n_mols)
      return fail(c, SHAPE_E_RANGE, "mol = %d outside [0, %d)", mol, M->n_mols);
    if (n < 0 || n > (1 << 24) || k0 < 0 || k0 > ((int64_t)1 << 62))
      return fail(c, SHAPE_E_RANGE, "need 0 <= n <= 2^24 and 0 <= k0 <= 2^62");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    shape::Prepared P;
    if ((rc = prepare(c, M, false, st, &P))) return rc;
    int bad = 0;
    HIP_TRY(c, hipMemcpyAsync(&bad, P.bad + mol, sizeof(int), hipMemcpyDeviceToHost, st),
            "copy");
    HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    if (bad) {
      HIP_TRY(c, shape::launch_fill_int(c->flag, 1, 0, st), "flag reset");
      return fail(c, SHAPE_E_DATA, "molecule %d is invalid data", mol);
    }
    const int anti = c->sampling == SHAPE_SAMPLING_ANTITHETIC ? 1 : 0;
    HIP_TRY(c, shape::launch_sample_points(P, M->atom_offset, mol, M->max_atoms, k0, n,
                                           key_of(seed), anti, thr, words, (int*)comp, r, st),
            "sample points kernel");
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_screen(shape_ctx* c, const shape_mols* query, const shape_mols* lib,
                 const int32_t* pairs, int32_t n_pairs, const shape_screen_params* prm,
                 void* stream, const shape_screen_out* out) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_screen");
  try {
    hipStream_t st = (hipStream_t)stream;
    shape::ScreenArgs a;
    int rc = screen_setup(c, query, lib, pairs, n_pairs, prm, st, out, &a);
    if (rc || a.n_pairs == 0) return rc;
    KernelTimer timer(c, st);
    HIP_TRY(c, shape::launch_screen(a, screen_variant_of(c), st), "screen kernel");
    timer.stop();
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

// Tuning cache: the variant shape_screen_tune chose for a kind of screen,
// process-wide (a variant suits any context on the same kind of device), and
// optionally appended to a text file from which a later process reads it.
}  // extern "C"

namespace {

std::mutex g_tune_m;
std::map<std::string, int> g_tune;
std::string g_tune_file;
constexpr const char* kTuneTag = "shape-tune-v1";

int floor_log2(int64_t x) {
  int b = -1;
  while (x > 0) {
    x >>= 1;
    ++b;
  }
  return b;
}

// The screen's kind: device (architecture, compute units), mode and
// sampling, the per-pair sample schedule, whether budgets are seeded, and the
// power-of-two classes of the pair count, the query's atom count and the
// library's mean atom count.
std::string tune_key(const shape_ctx* c, const shape_mols* query, const shape_mols* lib,
                     int32_t n_pairs, const shape_screen_params* prm) {
  const bool fixed = prm->mode == SHAPE_SCREEN_FIXED;
  char k[256];
  snprintf(k, sizeof k, "%s %d %d %d %d %d %d %d %d %d %d", c->arch, c->n_cu, prm->mode,
           c->sampling, fixed ? prm->n_per_side : 0, fixed ? 0 : prm->round_per_pair,
           fixed ? 0 : prm->cap_per_pair, (!fixed && prm->n_start) ? 1 : 0, floor_log2(n_pairs),
           floor_log2(query->max_atoms), floor_log2(lib->n_atoms / (lib->n_mols > 0 ? lib->n_mols : 1)));
  return k;
}

}  // namespace

extern "C" {

int shape_tune_cache_file(const char* path) {
  std::lock_guard<std::mutex> lock(g_tune_m);
  if (!path) {
    g_tune_file.clear();
    return SHAPE_OK;
  }
  if (!*path) return fail(nullptr, SHAPE_E_INVAL, "empty tuning-cache path");
  if (FILE* f = fopen(path, "r")) {
    char line[512];
    while (fgets(line, sizeof line, f)) {
      // tag, eleven key fields, variant; anything else is skipped
      char tag[32], arch[64];
      int v[10], variant;
      if (sscanf(line, "%31s %63s %d %d %d %d %d %d %d %d %d %d %d", tag, arch, &v[0], &v[1],
                 &v[2], &v[3], &v[4], &v[5], &v[6], &v[7], &v[8], &v[9], &variant) != 13 ||
          strcmp(tag, kTuneTag) != 0 || variant < 0 || variant >= shape::kScreenVariants)
        continue;
      char k[256];
      snprintf(k, sizeof k, "%s %d %d %d %d %d %d %d %d %d %d", arch, v[0], v[1], v[2], v[3],
               v[4], v[5], v[6], v[7], v[8], v[9]);
      g_tune[k] = variant;
    }
    fclose(f);
  } else if (FILE* w = fopen(path, "a")) {
    fclose(w);  // a new file: its directory is writable
  } else {
    return fail(nullptr, SHAPE_E_INVAL, "cannot open tuning cache %s", path);
  }
  g_tune_file = path;
  return SHAPE_OK;
}

int shape_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_m);
  g_tune.clear();
  return SHAPE_OK;
}

int32_t shape_tune_cache_size(void) {
  std::lock_guard<std::mutex> lock(g_tune_m);
  return (int32_t)g_tune.size();
}

int shape_screen_tune(shape_ctx* c, const shape_mols* query, const shape_mols* lib,
                      const int32_t* pairs, int32_t n_pairs, const shape_screen_params* prm,
                      void* stream, float* ms, int32_t* best) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_screen_tune");
  if (c->capturing) return refuse_in_capture(c, "shape_screen_tune");
  try {
    hipStream_t st = (hipStream_t)stream;
    void* scratch;
    int rc;
    if (n_pairs < 0) return fail(c, SHAPE_E_RANGE, "n_pairs < 0");
    if ((rc = ensure(c, S_TUNE, (size_t)(n_pairs > 0 ? n_pairs : 1) * 2 * sizeof(float),
                     &scratch)))
      return rc;
    shape_screen_out o{};
    o.T = (float*)scratch;
    o.se_T = (float*)scratch + (n_pairs > 0 ? n_pairs : 1);
    shape::ScreenArgs a;
    if ((rc = screen_setup(c, query, lib, pairs, n_pairs, prm, st, &o, &a))) return rc;
    float t[shape::kScreenVariants];
    int pick = 0;
    std::string key;
    if (a.n_pairs > 0) {
      key = tune_key(c, query, lib, n_pairs, prm);
      std::lock_guard<std::mutex> lock(g_tune_m);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {  // chosen before: no timing
        c->screen_variant = it->second;
        if (ms)
          for (int v = 0; v < shape::kScreenVariants; ++v) ms[v] = -1.0f;
        if (best) *best = it->second;
        return SHAPE_OK;
      }
    }
    if (a.n_pairs > 0) {
      hipEvent_t e0, e1;
      HIP_TRY(c, hipEventCreate(&e0), "hipEventCreate");
      hipError_t e = hipEventCreate(&e1);
      if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(c, e, "hipEventCreate");
      }
      e = shape::launch_screen(a, 0, st);  // warm-up
      for (int v = 0; v < shape::kScreenVariants && e == hipSuccess; ++v) {
        t[v] = 3.0e38f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
          float dt = 0.0f;
          e = hipEventRecord(e0, st);
          if (e == hipSuccess) e = shape::launch_screen(a, v, st);
          if (e == hipSuccess) e = hipEventRecord(e1, st);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          if (e == hipSuccess) e = hipEventElapsedTime(&dt, e0, e1);
          if (e == hipSuccess && dt < t[v]) t[v] = dt;
        }
        if (e == hipSuccess && t[v] < t[pick]) pick = v;
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (e != hipSuccess) return hip_fail(c, e, "screen tuning");
      std::lock_guard<std::mutex> lock(g_tune_m);
      g_tune[key] = pick;
      if (!g_tune_file.empty()) {
        if (FILE* f = fopen(g_tune_file.c_str(), "a")) {
          fprintf(f, "%s %s %d\n", kTuneTag, key.c_str(), pick);
          fclose(f);
        }
      }
    } else {
      for (int v = 0; v < shape::kScreenVariants; ++v) t[v] = 0.0f;
    }
    c->screen_variant = pick;
    if (ms)
      for (int v = 0; v < shape::kScreenVariants; ++v) ms[v] = t[v];
    if (best) *best = pick;
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_set_sampling(shape_ctx* c, int32_t sampling) {
  if (!c) return SHAPE_E_INVAL;
  if (sampling != SHAPE_SAMPLING_IID && sampling != SHAPE_SAMPLING_ANTITHETIC)
    return fail(c, SHAPE_E_INVAL, "unknown sampling %d", sampling);
  c->sampling = sampling;
  return SHAPE_OK;
}

int32_t shape_get_sampling(const shape_ctx* c) { return c ? c->sampling : -1; }

int shape_prepare_cache(shape_ctx* c, int enable) {
  if (!c) return SHAPE_E_INVAL;
  c->prep_cache = enable != 0;
  c->prepared[0].valid = false;
  c->prepared[1].valid = false;
  return SHAPE_OK;
}

int shape_screen_set_variant(shape_ctx* c, int32_t variant) {
  if (!c) return SHAPE_E_INVAL;
  if (variant < -1 || variant >= shape::kScreenVariants)
    return fail(c, SHAPE_E_RANGE, "variant %d outside [-1, %d)", variant,
                shape::kScreenVariants);
  c->screen_variant = variant;
  return SHAPE_OK;
}

int32_t shape_screen_get_variant(const shape_ctx* c) { return c ? c->screen_variant : -1; }

int shape_self_overlap(shape_ctx* c, const shape_mols* M, int32_t n_samples, uint64_t seed,
                       void* stream, float* O_self) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_self_overlap");
  try {
    int rc;
    if ((rc = check_mols(c, M, "M", false))) return rc;
    if (!O_self) return fail(c, SHAPE_E_INVAL, "O_self is NULL");
    if (n_samples < 2 || n_samples > (1 << 20))
      return fail(c, SHAPE_E_RANGE, "n_samples must lie in [2, 2^20]");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    shape::Prepared P;
    if ((rc = prepare(c, M, false, st, &P))) return rc;
    HIP_TRY(c, shape::launch_self_overlap(P, M->atom_offset, M->n_mols, n_samples, key_of(seed),
                                          O_self, st),
            "self-overlap kernel");
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

}  // extern "C"

namespace {

int align_check(shape_ctx* c, const shape_mols* A, const shape_mols* B, int32_t n_starts,
                int32_t n_samples) {
  int rc;
  if ((rc = check_mols(c, A, "A", false))) return rc;
  if ((rc = check_mols(c, B, "B", false))) return rc;
  if (A->n_mols != B->n_mols)
    return fail(c, SHAPE_E_RANGE, "A and B must hold the same number of molecules");
  if (n_starts < 1) return fail(c, SHAPE_E_RANGE, "n_starts < 1");
  if (n_samples < 64 || n_samples > 4096)
    return fail(c, SHAPE_E_RANGE, "n_samples must lie in [64, 4096]");
  const size_t lds = shape::align_lds_bytes(n_samples, A->max_atoms, B->max_atoms);
  if (lds > c->lds_per_block)
    return fail(c, SHAPE_E_RANGE, "alignment staging needs %zu B of LDS, device allows %zu",
                lds, c->lds_per_block);
  return SHAPE_OK;
}

int align_launch(shape_ctx* c, const shape_mols* A, const shape_mols* B,
                 const shape::Prepared& PA, const shape::Prepared& PB, int32_t n_starts,
                 const float* pose, const float* O_aa, const float* O_bb, int32_t n_samples,
                 uint64_t seed, hipStream_t st, float* T, float* grad,
                 const WorkOrder& wo) {
  if (wo.order)
    HIP_TRY(c, shape::launch_work_order(align_order_args(A, B, n_starts, 0), wo.order, wo.work,
                                        st),
            "launch order kernels");
  shape::AlignArgs a;
  a.A = PA;
  a.offA = A->atom_offset;
  a.max_a = A->max_atoms;
  a.B = PB;
  a.offB = B->atom_offset;
  a.max_b = B->max_atoms;
  a.n_starts = n_starts;
  a.n_samples = n_samples;
  a.key = key_of(seed);
  a.pose = pose;
  a.O_aa = O_aa;
  a.O_bb = O_bb;
  a.T = T;
  a.grad = grad;
  a.n_steps = 0;
  a.lr = 0.f;
  a.pose_out = nullptr;
  a.order = wo.order;
  HIP_TRY(c, shape::launch_align(a, A->n_mols, st), "alignment kernel");
  return SHAPE_OK;
}

}  // namespace

extern "C" {

int shape_align_grad(shape_ctx* c, const shape_mols* A, const shape_mols* B, int32_t n_starts,
                     const float* pose, const float* O_aa, const float* O_bb, int32_t n_samples,
                     uint64_t seed, void* stream, float* T, float* dT_dpose) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_align_grad");
  try {
    int rc;
    if ((rc = align_check(c, A, B, n_starts, n_samples))) return rc;
    if (!pose || !O_aa || !O_bb || !T) return fail(c, SHAPE_E_INVAL, "NULL array");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    WorkOrder wo;
    if ((rc = work_order_slot(c, A->n_mols, kOrderAlignPerCu, &wo))) return rc;
    shape::Prepared PA, PB;
    if ((rc = prepare(c, A, true, st, &PA))) return rc;
    if ((rc = prepare(c, B, false, st, &PB))) return rc;
    KernelTimer timer(c, st);
    rc = align_launch(c, A, B, PA, PB, n_starts, pose, O_aa, O_bb, n_samples, seed, st, T,
                      dT_dpose, wo);
    timer.stop();
    return rc;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_adam_pose(shape_ctx* c, float* pose, const float* dT_dpose, float* m, float* v,
                    int64_t n_poses, int32_t* step, float lr, float beta1, float beta2, float eps,
                    void* stream) {
  if (!c) return SHAPE_E_INVAL;
  if (n_poses < 0) return fail(c, SHAPE_E_RANGE, "n_poses < 0");
  if (n_poses == 0) return SHAPE_OK;
  if (!pose || !dT_dpose || !m || !v || !step) return fail(c, SHAPE_E_INVAL, "NULL array");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return fail(c, SHAPE_E_RANGE, "Adam hyper-parameters out of range");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, shape::launch_adam_pose(pose, dT_dpose, m, v, n_poses, step, lr, beta1, beta2, eps,
                                     (hipStream_t)stream),
          "Adam kernel");
  return SHAPE_OK;
}

int shape_align(shape_ctx* c, const shape_mols* A, const shape_mols* B, int32_t n_starts,
                float* pose, int32_t n_samples, int32_t n_steps, float lr, uint64_t seed,
                void* stream, float* T_final, int32_t* best) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_align");
  try {
    int rc;
    if ((rc = align_check(c, A, B, n_starts, n_samples))) return rc;
    if (!pose || !T_final) return fail(c, SHAPE_E_INVAL, "NULL array");
    if (n_steps < 0) return fail(c, SHAPE_E_RANGE, "n_steps < 0");
    if (!(lr > 0.f)) return fail(c, SHAPE_E_RANGE, "lr must be > 0");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int pairs = A->n_mols;
    shape::Prepared PA, PB;
    void *saa, *sbb;
    if ((rc = ensure(c, S_SELF_A, (size_t)pairs * sizeof(float), &saa))) return rc;
    if ((rc = ensure(c, S_SELF_B, (size_t)pairs * sizeof(float), &sbb))) return rc;
    WorkOrder wo;
    if ((rc = work_order_slot(c, pairs, kOrderAlignPerCu, &wo))) return rc;
    // self-overlaps use the library slots; prepare both sets afterwards
    if ((rc = prepare(c, A, false, st, &PB))) return rc;
    HIP_TRY(c, shape::launch_self_overlap(PB, A->atom_offset, pairs, n_samples, key_of(seed),
                                          (float*)saa, st),
            "self-overlap kernel");
    if ((rc = prepare(c, B, false, st, &PB))) return rc;
    HIP_TRY(c, shape::launch_self_overlap(PB, B->atom_offset, pairs, n_samples, key_of(seed),
                                          (float*)sbb, st),
            "self-overlap kernel");
    if ((rc = prepare(c, A, true, st, &PA))) return rc;
    // the whole optimisation in one launch: A's samples are drawn once per
    // pair, each start's Adam state stays in registers (the same steps as
    // shape_align_grad followed by shape_adam_pose, n_steps times)
    shape::AlignArgs a;
    a.A = PA;
    a.offA = A->atom_offset;
    a.max_a = A->max_atoms;
    a.B = PB;
    a.offB = B->atom_offset;
    a.max_b = B->max_atoms;
    a.n_starts = n_starts;
    a.n_samples = n_samples;
    a.key = key_of(seed);
    a.pose = pose;
    a.O_aa = (const float*)saa;
    a.O_bb = (const float*)sbb;
    a.T = T_final;
    a.grad = nullptr;
    a.n_steps = n_steps;
    a.lr = lr;
    a.pose_out = pose;
    a.order = wo.order;
    if (wo.order)
      HIP_TRY(c, shape::launch_work_order(align_order_args(A, B, n_starts, n_steps), wo.order,
                                          wo.work, st),
              "launch order kernels");
    KernelTimer timer(c, st);
    HIP_TRY(c, shape::launch_align(a, pairs, st), "alignment kernel");
    timer.stop();
    if (best) HIP_TRY(c, shape::launch_best_start(T_final, pairs, n_starts, best, st), "best");
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

// Pairs of the hybrid pipeline: B holds one molecule per pair, A one
// molecule per pair or a single molecule shared by all pairs.
int fo_pairs_check(shape_ctx* c, const shape_mols* A, const shape_mols* B) {
  int rc;
  if ((rc = check_mols(c, A, "A", false))) return rc;
  if ((rc = check_mols(c, B, "B", false))) return rc;
  if (A->n_mols != 1 && A->n_mols != B->n_mols)
    return fail(c, SHAPE_E_RANGE, "A->n_mols = %d must be 1 or B->n_mols = %d", A->n_mols,
                B->n_mols);
  return SHAPE_OK;
}

shape::MolsDev mols_dev(const shape_mols* m) {
  return shape::MolsDev{m->n_mols, m->max_atoms, m->n_atoms, m->atom_offset, m->xyz, m->alpha,
                        m->mol_id};
}

int shape_fo_starts(shape_ctx* c, const shape_mols* A, const shape_mols* B, int32_t n_random,
                    uint64_t seed, void* stream, float* pose) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_fo_starts");
  try {
    int rc;
    if ((rc = fo_pairs_check(c, A, B))) return rc;
    if (n_random < 0 || n_random > 1024) return fail(c, SHAPE_E_RANGE, "n_random outside [0, 1024]");
    if (!pose) return fail(c, SHAPE_E_INVAL, "pose is NULL");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    shape::Prepared PA, PB;
    if ((rc = prepare(c, A, true, st, &PA))) return rc;
    if ((rc = prepare(c, B, false, st, &PB))) return rc;
    HIP_TRY(c, shape::launch_fo_starts(mols_dev(A), mols_dev(B), PA.bad, PB.bad, n_random,
                                       key_of(seed), pose, st),
            "alignment starts kernel");
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_fo_align(shape_ctx* c, const shape_mols* A, const shape_mols* B, int32_t n_starts,
                   float* pose, int32_t n_steps, float lr, void* stream, float* T,
                   float* grad) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_fo_align");
  try {
    int rc;
    if ((rc = fo_pairs_check(c, A, B))) return rc;
    if (n_starts < 1) return fail(c, SHAPE_E_RANGE, "n_starts < 1");
    if ((int64_t)B->n_mols * n_starts > 0x7FFFFFFF)
      return fail(c, SHAPE_E_RANGE, "pairs x starts exceeds 2^31 - 1");
    if (n_steps < 0 || n_steps > 100000) return fail(c, SHAPE_E_RANGE, "n_steps outside [0, 1e5]");
    if (n_steps > 0 && !(lr > 0.f)) return fail(c, SHAPE_E_RANGE, "lr must be > 0");
    if (!pose || !T) return fail(c, SHAPE_E_INVAL, "pose and T are required");
    if (shape::fo_align_lds_bytes(A->max_atoms, B->max_atoms) > c->lds_per_block)
      return fail(c, SHAPE_E_RANGE, "molecules too large for the alignment kernel's LDS");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    WorkOrder wo;
    if (shape::fo_align_pair_major(A->max_atoms, B->max_atoms, n_starts) &&
        (rc = work_order_slot(c, B->n_mols, kOrderFoAlignPerCu, &wo)))
      return rc;
    shape::Prepared PA, PB;
    if ((rc = prepare(c, A, true, st, &PA))) return rc;
    if ((rc = prepare(c, B, false, st, &PB))) return rc;
    if (wo.order) {
      // per step and start: one pass over B's atoms (A's atoms sit on the
      // lanes) and the rotation, sums and Adam step, worth about 4 atoms
      shape::OrderArgs o{};
      o.n = B->n_mols;
      o.per_xcd = 1;
      o.offB = B->atom_offset;
      o.nB_mols = B->n_mols;
      o.max_b = B->max_atoms;
      o.wB = 1;
      o.w0 = 4;
      HIP_TRY(c, shape::launch_work_order(o, wo.order, wo.work, st), "launch order kernels");
    }
    KernelTimer timer(c, st);
    HIP_TRY(c, shape::launch_fo_align(mols_dev(A), mols_dev(B), PA.bad, PB.bad, n_starts,
                                      n_steps, lr, pose, T, grad, st, wo.order),
            "first-order alignment kernel");
    timer.stop();
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_best_pose(shape_ctx* c, int32_t n_pairs, int32_t n_starts, const float* T,
                    const float* pose, void* stream, float* best_pose, float* best_T) {
  if (!c) return SHAPE_E_INVAL;
  if (n_pairs < 0 || n_starts < 1) return fail(c, SHAPE_E_RANGE, "n_pairs < 0 or n_starts < 1");
  if (n_pairs == 0) return SHAPE_OK;
  if (!T || !pose || !best_pose) return fail(c, SHAPE_E_INVAL, "NULL array");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, shape::launch_best_pose(T, pose, n_pairs, n_starts, best_pose, best_T,
                                     (hipStream_t)stream),
          "best pose kernel");
  return SHAPE_OK;
}

int shape_group_max(shape_ctx* c, const float* T, int64_t n_T, const int32_t* group_offset,
                    int32_t n_groups, void* stream, float* best_T, int32_t* best_idx) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_group_max");
  if (n_groups < 0 || n_T < 0) return fail(c, SHAPE_E_RANGE, "n_groups < 0 or n_T < 0");
  if (n_groups == 0) return SHAPE_OK;
  if (!group_offset || !best_T || (n_T > 0 && !T)) return fail(c, SHAPE_E_INVAL, "NULL array");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, shape::launch_group_max(T, n_T, group_offset, n_groups, best_T, best_idx, c->flag,
                                     (hipStream_t)stream),
          "group max kernel");
  return SHAPE_OK;
}

int shape_apply_pose(shape_ctx* c, const shape_mols* M, const float* pose, void* stream,
                     float* xyz_out) {
  if (!c) return SHAPE_E_INVAL;
  int rc;
  if ((rc = check_mols(c, M, "M", false))) return rc;
  if (!pose || !xyz_out) return fail(c, SHAPE_E_INVAL, "NULL array");
  if ((rc = set_device(c))) return rc;
  HIP_TRY(c, shape::launch_apply_pose(mols_dev(M), pose, xyz_out, (hipStream_t)stream),
          "apply pose kernel");
  return SHAPE_OK;
}

int shape_grid_integrals(shape_ctx* c, const shape_mols* A, const shape_mols* B, double h,
                         double pad, void* stream, double* out8) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_grid_integrals");
  if (c->capturing) return refuse_in_capture(c, "shape_grid_integrals");
  try {
    int rc;
    if ((rc = check_mols(c, A, "A", true))) return rc;
    if ((rc = check_mols(c, B, "B", true))) return rc;
    if (!out8) return fail(c, SHAPE_E_INVAL, "out is NULL");
    if (!(h > 0.0) || !isfinite(h) || !(pad >= 0.0) || !isfinite(pad))
      return fail(c, SHAPE_E_RANGE, "h must be > 0 and pad >= 0 (finite)");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    // invalid molecules are reported before the grid reads them
    shape::Prepared PA, PB;
    if ((rc = prepare(c, A, true, st, &PA))) return rc;
    if ((rc = prepare(c, B, false, st, &PB))) return rc;
    int bad[2] = {0, 0}, offA[2] = {0, 0}, offB[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(&bad[0], PA.bad, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
    HIP_TRY(c, hipMemcpyAsync(&bad[1], PB.bad, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
    HIP_TRY(c, hipMemcpyAsync(offA, A->atom_offset, sizeof offA, hipMemcpyDeviceToHost, st),
            "copy");
    HIP_TRY(c, hipMemcpyAsync(offB, B->atom_offset, sizeof offB, hipMemcpyDeviceToHost, st),
            "copy");
    HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    if (bad[0] || bad[1]) {
      HIP_TRY(c, shape::launch_fill_int(c->flag, 1, 0, st), "flag reset");
      return fail(c, SHAPE_E_DATA, "invalid molecule data in %s", bad[0] ? "A" : "B");
    }
    // the preparation has validated both ranges
    const int na = offA[1] - offA[0], nb = offB[1] - offB[0];
    const float* xa = A->xyz + 3 * (size_t)offA[0];
    const float* aa = A->alpha + offA[0];
    const float* xb = B->xyz + 3 * (size_t)offB[0];
    const float* ab = B->alpha + offB[0];
    void *box_d, *tab, *part;
    if ((rc = ensure(c, S_GRID_BOX, 16 * sizeof(double), &box_d))) return rc;
    HIP_TRY(c, shape::launch_grid_box(xa, na, xb, nb, (double*)box_d, st), "grid box");
    double box[6];
    HIP_TRY(c, hipMemcpyAsync(box, box_d, sizeof box, hipMemcpyDeviceToHost, st), "copy");
    HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    shape::GridDims g;
    g.h = h;
    g.nmax = 0;
    int64_t points = 1;
    for (int d = 0; d < 3; ++d) {
      g.lo[d] = box[d] - pad;
      const double hi = box[3 + d] + pad;
      const double nd = ceil((hi - g.lo[d]) / h) + 1.0;
      if (nd > 65536.0) return fail(c, SHAPE_E_RANGE, "grid exceeds 65,536 points per axis");
      g.n[d] = (int)nd;
      g.nmax = g.n[d] > g.nmax ? g.n[d] : g.nmax;
      points *= g.n[d];
    }
    if (points > ((int64_t)1 << 36)) return fail(c, SHAPE_E_RANGE, "grid exceeds 2^36 points");
    const int64_t cols = (int64_t)g.n[0] * g.n[1];
    if (cols > 0x7FFFFFFF) return fail(c, SHAPE_E_RANGE, "grid has too many columns");
    const size_t lds = (size_t)(na + nb) * sizeof(double);
    if (lds + 8 * 4 * sizeof(double) > c->lds_per_block)
      return fail(c, SHAPE_E_RANGE, "molecules too large for the grid kernel's LDS");
    if ((rc = ensure(c, S_GRID_TAB, (size_t)3 * (na + nb) * g.nmax * sizeof(double), &tab)))
      return rc;
    if ((rc = ensure(c, S_GRID_PART, (size_t)cols * 8 * sizeof(double), &part))) return rc;
    KernelTimer timer(c, st);
    HIP_TRY(c, shape::launch_grid(xa, aa, na, xb, ab, nb, g, (double*)tab, (double*)part,
                                  (double*)box_d + 8, st),
            "grid kernels");
    timer.stop();
    HIP_TRY(c, hipMemcpyAsync(out8, (double*)box_d + 8, 8 * sizeof(double),
                              hipMemcpyDeviceToHost, st),
            "result copy");
    HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_features(shape_ctx* c, const shape_mols* M, void* stream, float* out) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_features");
  try {
    int rc;
    if ((rc = check_mols(c, M, "M", false))) return rc;
    if (!out) return fail(c, SHAPE_E_INVAL, "out is NULL");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    void* mom;
    if ((rc = ensure(c, S_FEAT_MOM, (size_t)M->n_mols * 6 * sizeof(float), &mom))) return rc;
    WorkOrder wo;
    if ((rc = work_order_slot(c, M->n_mols, kOrderFeaturesPerCu, &wo))) return rc;
    KernelTimer timer(c, st);
    if (wo.order) {
      // molecules by descending squared atom count (the overlap triangle)
      shape::OrderArgs o{};
      o.n = M->n_mols;
      o.offB = M->atom_offset;
      o.nB_mols = M->n_mols;
      o.max_b = M->max_atoms;
      o.quad_b = 1;
      o.wB = 1;
      o.w0 = 64;
      HIP_TRY(c, shape::launch_work_order(o, wo.order, wo.work, st), "features launch order");
    }
    HIP_TRY(c, shape::launch_features(mols_dev(M), c->flag, out, (float*)mom, st, wo.order),
            "features kernel");
    timer.stop();
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_fo_overlap(shape_ctx* c, const shape_mols* query, const shape_mols* lib,
                     const int32_t* pairs, int32_t n_pairs, void* stream, float* out) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_fo_overlap");
  try {
    int rc;
    if ((rc = check_mols(c, query, "query", true))) return rc;
    if ((rc = check_mols(c, lib, "lib", false))) return rc;
    if (n_pairs < 0) return fail(c, SHAPE_E_RANGE, "n_pairs < 0");
    if (!pairs && n_pairs > lib->n_mols)
      return fail(c, SHAPE_E_RANGE, "n_pairs exceeds lib->n_mols");
    if (n_pairs == 0) return SHAPE_OK;
    if (!out) return fail(c, SHAPE_E_INVAL, "out is NULL");
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, shape::launch_fo_cross(mols_dev(query), mols_dev(lib), pairs, n_pairs, c->n_cu,
                                      c->flag, out, st),
            "first-order overlap kernel");
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_pair_features(shape_ctx* c, const float* f_q, const float* f_lib, const int32_t* qidx,
                        const int32_t* idx, int32_t n, const float* fo_cross, const float* mean,
                        const float* inv_std, void* stream, float* out) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_pair_features");
  if (n < 0) return fail(c, SHAPE_E_RANGE, "n < 0");
  if (n == 0) return SHAPE_OK;
  if (!f_q || !f_lib || !mean || !inv_std || !out) return fail(c, SHAPE_E_INVAL, "NULL array");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, shape::launch_pair_features(f_q, f_lib, qidx, idx, n, fo_cross, mean, inv_std,
                                         out, (hipStream_t)stream),
          "pair features kernel");
  return SHAPE_OK;
}

int shape_mlp_infer(shape_ctx* c, const float* f_q, const float* f_lib, const int32_t* qidx,
                    const int32_t* idx, int32_t n, const float* fo_cross, const float* mean,
                    const float* inv_std, const float* params, void* stream, float* out) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_mlp_infer");
  try {
    if (n < 0) return fail(c, SHAPE_E_RANGE, "n < 0");
    if (n == 0) return SHAPE_OK;
    if (!f_q || !f_lib || !mean || !inv_std || !params || !out)
      return fail(c, SHAPE_E_INVAL, "NULL array");
    int rc = set_device(c);
    if (rc) return rc;
    void* packed;
    if ((rc = ensure(c, S_MLP_PACK, shape::mlp_pack_bytes(), &packed))) return rc;
    KernelTimer timer(c, (hipStream_t)stream);
    HIP_TRY(c, shape::launch_mlp_infer(f_q, f_lib, qidx, idx, n, fo_cross, mean, inv_std, params,
                                       packed, out, (hipStream_t)stream),
            "surrogate inference kernel");
    timer.stop();
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_mlp_forward(shape_ctx* c, const float* f_q, const float* f_lib, const int32_t* qidx,
                      const int32_t* idx, int32_t n, const float* fo_cross, const float* mean,
                      const float* inv_std, const float* params, void* stream, float* x,
                      float* h1, float* h2, float* h3, float* out) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_mlp_forward");
  try {
    if (n < 0) return fail(c, SHAPE_E_RANGE, "n < 0");
    if (n == 0) return SHAPE_OK;
    if (!f_q || !f_lib || !mean || !inv_std || !params || !out || !x || !h1 || !h2 || !h3)
      return fail(c, SHAPE_E_INVAL, "NULL array");
    if ((((uintptr_t)x) | ((uintptr_t)h1) | ((uintptr_t)h2) | ((uintptr_t)h3)) & 15u)
      return fail(c, SHAPE_E_INVAL, "x, h1, h2, h3 must be 16-byte aligned");
    int rc = set_device(c);
    if (rc) return rc;
    void* packed;
    if ((rc = ensure(c, S_MLP_PACK, shape::mlp_pack_bytes(), &packed))) return rc;
    float* const h[3] = {h1, h2, h3};
    KernelTimer timer(c, (hipStream_t)stream);
    HIP_TRY(c, shape::launch_mlp_infer(f_q, f_lib, qidx, idx, n, fo_cross, mean, inv_std, params,
                                       packed, out, (hipStream_t)stream, x, h),
            "surrogate forward kernel");
    timer.stop();
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_seed_budget(shape_ctx* c, const float* raw, int64_t ld, const int32_t* idx, int32_t k,
                      double y_mean, double y_std, double tau, int32_t round_per_pair,
                      int32_t cap_per_pair, void* stream, int32_t* n_start) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_seed_budget");
  if (k < 0) return fail(c, SHAPE_E_RANGE, "k < 0");
  if (k == 0) return SHAPE_OK;
  if (!raw || !n_start) return fail(c, SHAPE_E_INVAL, "NULL array");
  if (ld < 2) return fail(c, SHAPE_E_RANGE, "ld must be >= 2");
  if (!(tau > 0.0) || !isfinite(tau) || !isfinite(y_mean) || !isfinite(y_std))
    return fail(c, SHAPE_E_RANGE, "tau, y_mean, y_std must be finite (tau > 0)");
  if (round_per_pair < 1 || cap_per_pair < round_per_pair)
    return fail(c, SHAPE_E_RANGE, "need 1 <= round_per_pair <= cap_per_pair");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, shape::launch_seed_budget(raw, ld, idx, k, y_mean, y_std, tau, round_per_pair,
                                       cap_per_pair, n_start, (hipStream_t)stream),
          "seed budget kernel");
  return SHAPE_OK;
}

int shape_gemm(shape_ctx* c, int32_t M, int32_t N, int32_t K, const float* A, int64_t sam,
               int64_t sak, const float* B, int64_t sbk, int64_t sbn, float* C, int64_t scm,
               const float* bias, const float* gate, int64_t sgm, uint32_t flags, void* stream) {
  if (!c) return SHAPE_E_INVAL;
  if (M < 1 || N < 1 || K < 1) return fail(c, SHAPE_E_RANGE, "M, N, K must be >= 1");
  if (!A || !B || !C) return fail(c, SHAPE_E_INVAL, "NULL array");
  if (flags & ~(SHAPE_GEMM_BF16 | SHAPE_GEMM_RELU)) return fail(c, SHAPE_E_INVAL, "bad flags");
  int rc = set_device(c);
  if (rc) return rc;
  shape::GemmArgs g{M, N, K, A, sam, sak, B, sbk, sbn, C, scm, bias, gate, sgm, (int)flags};
  const int splits = shape::gemm_splits(g);
  if (splits > 1) {
    void* part;
    if ((rc = ensure(c, S_GEMM_PART, (size_t)splits * M * N * sizeof(float), &part))) return rc;
    g.part = (float*)part;
  }
  HIP_TRY(c, shape::launch_gemm(g, (hipStream_t)stream), "gemm kernel");
  return SHAPE_OK;
}

int shape_gemm_set(shape_ctx* c, int32_t n, const shape_gemm_desc* d, void* stream) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_gemm_set");
  if (n < 1 || n > shape::kGemmSetMax)
    return fail(c, SHAPE_E_RANGE, "n must be in 1..%d", shape::kGemmSetMax);
  if (!d) return fail(c, SHAPE_E_INVAL, "NULL descriptor array");
  try {
    shape::GemmArgs set[shape::kGemmSetMax];
    int n_set = 0;
    size_t part_elems = 0;
    int64_t set_blocks = 0;  // one grid: at most 2^31 - 1 workgroups
    for (int t = 0; t < n; ++t) {
      const shape_gemm_desc& q = d[t];
      if (q.M < 1 || q.N < 1 || q.K < 1) return fail(c, SHAPE_E_RANGE, "M, N, K must be >= 1");
      if (!q.A || !q.B || !q.C) return fail(c, SHAPE_E_INVAL, "NULL array");
      if (q.flags & ~(SHAPE_GEMM_BF16 | SHAPE_GEMM_RELU))
        return fail(c, SHAPE_E_INVAL, "bad flags");
    }
    int rc = set_device(c);
    if (rc) return rc;
    for (int t = 0; t < n; ++t) {
      const shape_gemm_desc& q = d[t];
      shape::GemmArgs g{q.M,   q.N,   q.K,    q.A,    q.sam,  q.sak,  q.B,         q.sbk,
                        q.sbn, q.C,   q.scm,  q.bias, q.gate, q.sgm,  (int)q.flags};
      if (shape::gemm_set_fits(g) && set_blocks + shape::gemm_set_blocks(g) <= 0x7FFFFFFF) {
        set[n_set++] = g;
        part_elems += shape::gemm_set_part_elems(g);
        set_blocks += shape::gemm_set_blocks(g);
      } else if ((rc = shape_gemm(c, q.M, q.N, q.K, q.A, q.sam, q.sak, q.B, q.sbk, q.sbn, q.C,
                                  q.scm, q.bias, q.gate, q.sgm, q.flags, stream))) {
        return rc;
      }
    }
    if (n_set == 0) return SHAPE_OK;
    void* part = nullptr;
    if (part_elems > 0 &&
        (rc = ensure(c, S_GEMM_PART, part_elems * sizeof(float), &part)))
      return rc;
    HIP_TRY(c, shape::launch_gemm_set(n_set, set, (float*)part, (hipStream_t)stream),
            "gemm set kernels");
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_mlp_pack(shape_ctx* c, const float* params, void* stream, void* packed) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_mlp_pack");
  if (!params || !packed) return fail(c, SHAPE_E_INVAL, "NULL array");
  if ((uintptr_t)packed & 15u) return fail(c, SHAPE_E_INVAL, "packed must be 16-byte aligned");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, shape::launch_mlp_pack_all(params, packed, (hipStream_t)stream), "packing kernels");
  return SHAPE_OK;
}

int shape_mlp_train_step(shape_ctx* c, const float* f_q, const float* f_lib, const int32_t* qidx,
                         const int32_t* idx, int32_t n, const float* fo_cross, const float* mean,
                         const float* inv_std, const float* target, const float* loss_w,
                         const shape_mlp_adam* opt, void* stream, float* grad, float* loss) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_mlp_train_step");
  try {
    const int rows = shape::mlp_step_rows();
    if (n < rows || n > SHAPE_MLP_STEP_MAX_ROWS || n % rows)
      return fail(c, SHAPE_E_RANGE, "n = %d: the fused step takes a multiple of %d rows in "
                  "[%d, %d]", n, rows, rows, SHAPE_MLP_STEP_MAX_ROWS);
    if (!f_q || !f_lib || !mean || !inv_std || !target || !loss_w || !opt || !loss)
      return fail(c, SHAPE_E_INVAL, "NULL array");
    if (!opt->params || !opt->m || !opt->v || !opt->step || !opt->packed)
      return fail(c, SHAPE_E_INVAL, "NULL optimiser array");
    if (((uintptr_t)opt->packed | (uintptr_t)opt->params) & 15u)
      return fail(c, SHAPE_E_INVAL, "packed and params must be 16-byte aligned");
    if (!(opt->lr > 0.f) || !(opt->beta1 >= 0.f && opt->beta1 < 1.f) ||
        !(opt->beta2 >= 0.f && opt->beta2 < 1.f) || !(opt->eps > 0.f))
      return fail(c, SHAPE_E_RANGE, "Adam hyper-parameters out of range");
    int rc = set_device(c);
    if (rc) return rc;
    void* scratch;
    if ((rc = ensure(c, S_MLP_STEP, shape::mlp_step_scratch_bytes(n), &scratch))) return rc;
    shape::MlpStep s{};
    s.fq = f_q;
    s.flib = f_lib;
    s.qidx = qidx;
    s.idx = idx;
    s.n = n;
    s.fo_cross = fo_cross;
    s.mean = mean;
    s.inv_std = inv_std;
    s.target = target;
    s.lw = loss_w;
    s.params = opt->params;
    s.m = opt->m;
    s.v = opt->v;
    s.step = opt->step;
    s.packed = opt->packed;
    s.lr = opt->lr;
    s.b1 = opt->beta1;
    s.b2 = opt->beta2;
    s.eps = opt->eps;
    s.grad = grad;
    s.loss = loss;
    KernelTimer timer(c, (hipStream_t)stream);
    HIP_TRY(c, shape::launch_mlp_step(s, scratch, (hipStream_t)stream), "training step kernels");
    timer.stop();
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_mlp_backward(shape_ctx* c, int32_t n_layers, const int32_t* width, int32_t batch,
                       const float* params, const float* const* act, const float* dout,
                       uint32_t flags, void* stream, float* grad) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_mlp_backward");
  try {
    if (n_layers < 1 || n_layers > shape::kGemmSetMax)
      return fail(c, SHAPE_E_RANGE, "n_layers must be in 1..%d", shape::kGemmSetMax);
    if (batch < 1) return fail(c, SHAPE_E_RANGE, "batch < 1");
    if (!width || !params || !act || !dout || !grad) return fail(c, SHAPE_E_INVAL, "NULL array");
    if (flags & ~SHAPE_GEMM_BF16) return fail(c, SHAPE_E_INVAL, "bad flags");
    int64_t d_elems = 0;
    for (int l = 0; l <= n_layers; ++l) {
      if (width[l] < 1 || width[l] > 65536)
        return fail(c, SHAPE_E_RANGE, "width[%d] = %d outside [1, 65536]", l, width[l]);
      if (l < n_layers && !act[l]) return fail(c, SHAPE_E_INVAL, "act[%d] is NULL", l);
      if (l >= 1 && l < n_layers) d_elems += (int64_t)batch * width[l];
    }
    int rc = set_device(c);
    if (rc) return rc;
    // gradients w.r.t. the hidden layers' outputs, through their ReLUs: kept
    // until the weight-gradient products below have read them
    void* dbuf = nullptr;
    if (d_elems > 0 &&
        (rc = ensure(c, S_MLP_D, (size_t)d_elems * sizeof(float), &dbuf)))
      return rc;
    int64_t off[shape::kGemmSetMax + 1];
    off[0] = 0;
    for (int l = 0; l < n_layers; ++l)
      off[l + 1] = off[l] + (int64_t)width[l] * width[l + 1] + width[l + 1];
    int64_t d_off[shape::kGemmSetMax];
    int64_t o = 0;
    for (int l = 1; l < n_layers; ++l) {
      d_off[l] = o;
      o += (int64_t)batch * width[l];
    }
    shape_gemm_desc wg[shape::kGemmSetMax];
    int32_t cM[shape::kColSetMax], cN[shape::kColSetMax];
    const float* cA[shape::kColSetMax];
    int64_t cld[shape::kColSetMax];
    float* cout_[shape::kColSetMax];
    const float* dz = dout;
    int n = 0;
    for (int l = n_layers - 1; l >= 0; --l, ++n) {
      const int n_in = width[l], n_out = width[l + 1];
      // dW[i][o] = sum_b act[l][b][i] dz[b][o]; db[o] = sum_b dz[b][o]
      shape_gemm_desc& d = wg[n];
      d = shape_gemm_desc{};
      d.A = act[l];
      d.sam = 1;
      d.sak = n_in;
      d.B = dz;
      d.sbk = n_out;
      d.sbn = 1;
      d.C = grad + off[l];
      d.scm = n_out;
      d.M = n_in;
      d.N = n_out;
      d.K = batch;
      d.flags = flags;
      cM[n] = batch;
      cN[n] = n_out;
      cA[n] = dz;
      cld[n] = n_out;
      cout_[n] = grad + off[l] + (int64_t)n_in * n_out;
      if (l > 0) {
        // dh[b][i] = sum_o dz[b][o] W[i][o], zero where the ReLU was off
        float* dn = (float*)dbuf + d_off[l];
        if ((rc = shape_gemm(c, batch, n_in, n_out, dz, n_out, 1, params + off[l], 1, n_out, dn,
                             n_in, nullptr, act[l], n_in, flags, stream)))
          return rc;
        dz = dn;
      }
    }
    if ((rc = shape_gemm_set(c, n, wg, stream))) return rc;
    return shape_colsum_set(c, n, cM, cN, cA, cld, cout_, stream);
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_colsum(shape_ctx* c, int32_t M, int32_t N, const float* A, int64_t lda, float* out,
                 void* stream) {
  if (!c) return SHAPE_E_INVAL;
  if (M < 1 || N < 1) return fail(c, SHAPE_E_RANGE, "M, N must be >= 1");
  if (!A || !out) return fail(c, SHAPE_E_INVAL, "NULL array");
  int rc = set_device(c);
  if (rc) return rc;
  void* part;
  if ((rc = ensure(c, S_COLSUM, (size_t)shape::colsum_chunks(M) * N * sizeof(float), &part)))
    return rc;
  HIP_TRY(c, shape::launch_colsum(A, M, N, lda, (float*)part, out, (hipStream_t)stream),
          "colsum kernels");
  return SHAPE_OK;
}

int shape_colsum_set(shape_ctx* c, int32_t n_mats, const int32_t* M, const int32_t* N,
                     const float* const* A, const int64_t* lda, float* const* out,
                     void* stream) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_colsum_set");
  if (n_mats < 1 || n_mats > shape::kColSetMax)
    return fail(c, SHAPE_E_RANGE, "n_mats must be in 1..%d", shape::kColSetMax);
  if (!M || !N || !A || !lda || !out) return fail(c, SHAPE_E_INVAL, "NULL array");
  int64_t blocks = 0;
  for (int t = 0; t < n_mats; ++t) {
    if (M[t] < 1 || N[t] < 1) return fail(c, SHAPE_E_RANGE, "M, N must be >= 1");
    if (!A[t] || !out[t]) return fail(c, SHAPE_E_INVAL, "NULL array");
    blocks += (N[t] + 15) / 16;
  }
  if (blocks > 0x7FFFFFFF) return fail(c, SHAPE_E_RANGE, "too many columns");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, shape::launch_colsum_set(n_mats, M, N, A, lda, out, (hipStream_t)stream),
          "colsum kernel");
  return SHAPE_OK;
}

int shape_mse(shape_ctx* c, int32_t B, int32_t N, const float* y, const float* t, const float* w,
              void* stream, float* grad, float* loss) {
  if (!c) return SHAPE_E_INVAL;
  if (B < 1 || N < 1) return fail(c, SHAPE_E_RANGE, "B, N must be >= 1");
  if (!y || !t || !w || !grad || !loss) return fail(c, SHAPE_E_INVAL, "NULL array");
  int rc = set_device(c);
  if (rc) return rc;
  void* part;
  if ((rc = ensure(c, S_MSE, (size_t)shape::mse_blocks(B, N) * sizeof(double), &part))) return rc;
  HIP_TRY(c, shape::launch_mse(y, t, w, B, N, grad, (double*)part, loss, (hipStream_t)stream),
          "mse kernels");
  return SHAPE_OK;
}

int shape_adam(shape_ctx* c, float* p, const float* g, float* m, float* v, int64_t n,
               int32_t* step, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!c) return SHAPE_E_INVAL;
  if (n < 0) return fail(c, SHAPE_E_RANGE, "n < 0");
  if (n == 0) return SHAPE_OK;
  if (!p || !g || !m || !v || !step) return fail(c, SHAPE_E_INVAL, "NULL array");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return fail(c, SHAPE_E_RANGE, "Adam hyper-parameters out of range");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, shape::launch_adam(p, g, m, v, n, step, lr, beta1, beta2, eps, (hipStream_t)stream),
          "Adam kernel");
  return SHAPE_OK;
}

int shape_topk(shape_ctx* c, const float* score, int32_t n, int32_t k, void* stream,
               int32_t* idx) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_topk");
  if (n < 1 || k < 1 || k > n) return fail(c, SHAPE_E_RANGE, "need 1 <= k <= n");
  if (!score || !idx) return fail(c, SHAPE_E_INVAL, "NULL array");
  int rc = set_device(c);
  if (rc) return rc;
  void *sel, *hist, *gt, *eq;
  const int nb = shape::topk_blocks(n);
  if ((rc = ensure(c, S_TOPK_SEL, 4 * sizeof(uint32_t), &sel))) return rc;
  if ((rc = ensure(c, S_TOPK_HIST, 256 * sizeof(uint32_t), &hist))) return rc;
  if ((rc = ensure(c, S_TOPK_GT, (size_t)nb * sizeof(int), &gt))) return rc;
  if ((rc = ensure(c, S_TOPK_EQ, (size_t)nb * sizeof(int), &eq))) return rc;
  KernelTimer timer(c, (hipStream_t)stream);
  HIP_TRY(c, shape::launch_topk(score, n, k, (uint32_t*)sel, (uint32_t*)hist, (int*)gt, (int*)eq,
                                idx, (hipStream_t)stream),
          "top-k kernels");
  timer.stop();
  return SHAPE_OK;
}

int shape_peak_rates(shape_ctx* c, void* stream, double* rates) {
  if (!c) return SHAPE_E_INVAL;
  if (c->capturing) return refuse_in_capture(c, "shape_peak_rates");
  if (!rates) return fail(c, SHAPE_E_INVAL, "rates is NULL");
  try {
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int lanes = shape::peak_blocks(c->n_cu) * 256;
    void* out;
    if ((rc = ensure(c, S_PEAK, (size_t)lanes * sizeof(float), &out))) return rc;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0), "hipEventCreate");
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      return hip_fail(c, e, "hipEventCreate");
    }
    // loop counts that keep each kernel busy for about a millisecond or more
    const int iters[5] = {16384, 4096, 8192, 2048, 8192};
    for (int w = 0; w < 5 && e == hipSuccess; ++w) {
      float best = 3.0e38f;
      e = shape::launch_peak(w, c->n_cu, 64, (float*)out, st);  // warm-up
      for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        float ms = 0.0f;
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) e = shape::launch_peak(w, c->n_cu, iters[w], (float*)out, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms < best) best = ms;
      }
      if (e == hipSuccess)
        rates[w] = (double)lanes * iters[w] * shape::peak_work_per_iter(w) / (best * 1e-3);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(c, e, "peak kernels");
    return SHAPE_OK;
  } catch (...) {
    return fail(c, SHAPE_E_HIP, "internal error");
  }
}

int shape_fail_allocations(shape_ctx* c, int32_t n) {
  if (!c) return SHAPE_E_INVAL;
  if (n < 0) return fail(c, SHAPE_E_RANGE, "n < 0");
  c->fail_allocs = n;
  return SHAPE_OK;
}

int shape_range_push(const char* name) {
  if (!name) return fail(nullptr, SHAPE_E_INVAL, "range name is NULL");
  roctxRangePushA(name);
  return SHAPE_OK;
}

int shape_range_pop(void) {
  roctxRangePop();
  return SHAPE_OK;
}

int shape_timing_enable(shape_ctx* c, int enable) {
  if (!c) return SHAPE_E_INVAL;
  c->timing = enable != 0;
  return SHAPE_OK;
}

int shape_timing_read(shape_ctx* c, double* total_ms, int64_t* launches, int reset) {
  if (c && c->capturing) return refuse_in_capture(c, "shape_timing_read");
  if (!c) return SHAPE_E_INVAL;
  int rc = set_device(c);
  if (rc) return rc;
  double sum = 0.0;
  for (auto& e : c->events) {
    HIP_TRY(c, hipEventSynchronize(e.second), "hipEventSynchronize");
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, e.first, e.second), "hipEventElapsedTime");
    sum += ms;
  }
  if (total_ms) *total_ms = sum;
  if (launches) *launches = (int64_t)c->events.size();
  if (reset) {
    for (auto& e : c->events) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    c->events.clear();
  }
  return SHAPE_OK;
}

int shape_check_data(shape_ctx* c, void* stream) {
  if (c && c->capturing) return refuse_in_capture(c, "shape_check_data");
  if (!c) return SHAPE_E_INVAL;
  int rc = set_device(c);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  int flag = 0;
  HIP_TRY(c, hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
  HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
  if (flag) {
    HIP_TRY(c, shape::launch_fill_int(c->flag, 1, 0, st), "flag reset");
    HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    return fail(c, SHAPE_E_DATA, "invalid molecule data seen since the last check");
  }
  return SHAPE_OK;
}

int shape_graph_begin(shape_ctx* c, void* stream) {
  if (!c) return SHAPE_E_INVAL;
  if (!stream) return fail(c, SHAPE_E_INVAL, "the null stream cannot be captured");
  if (c->capturing) return fail(c, SHAPE_E_UNSUPPORTED, "a graph capture is already open");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeRelaxed),
          "hipStreamBeginCapture");
  c->capturing = true;
  c->capture_failed = false;
  c->capture_stream = (hipStream_t)stream;
  // a preparation done before the capture is not part of the graph, and one
  // recorded inside it does not run now: neither may be reused across the
  // capture boundary
  c->prepared[0].valid = false;
  c->prepared[1].valid = false;
  return SHAPE_OK;
}

int shape_graph_end(shape_ctx* c, void* stream, shape_graph** out) {
  if (!c) return SHAPE_E_INVAL;
  if (out) *out = nullptr;
  if (!c->capturing || c->capture_stream != (hipStream_t)stream)
    return fail(c, SHAPE_E_INVAL, "no graph capture is open on this stream");
  c->capturing = false;
  c->capture_stream = nullptr;
  c->prepared[0].valid = false;
  c->prepared[1].valid = false;
  hipGraph_t g = nullptr;
  HIP_TRY(c, hipStreamEndCapture((hipStream_t)stream, &g), "hipStreamEndCapture");
  if (c->capture_failed) {
    (void)hipGraphDestroy(g);
    return fail(c, SHAPE_E_UNSUPPORTED, "a call failed during capture (capture discarded): %s",
                c->err.c_str());
  }
  if (!out) {
    (void)hipGraphDestroy(g);
    return fail(c, SHAPE_E_INVAL, "out is NULL (capture discarded)");
  }
  shape_graph* sg = new (std::nothrow) shape_graph();
  if (!sg) {
    (void)hipGraphDestroy(g);
    return fail(c, SHAPE_E_NOMEM, "graph allocation failed");
  }
  hipError_t e = hipGraphInstantiate(&sg->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    delete sg;
    return hip_fail(c, e, "hipGraphInstantiate");
  }
  sg->device = c->device;
  sg->life = c->life;
  {
    std::lock_guard<std::mutex> lk(c->life->m);
    ++c->life->live;
  }
  *out = sg;
  return SHAPE_OK;
}

int shape_graph_launch(shape_ctx* c, shape_graph* g, void* stream) {
  if (!c) return SHAPE_E_INVAL;
  ProfRange range_("shape_graph_launch");
  if (!g || !g->exec) return fail(c, SHAPE_E_INVAL, "graph is NULL");
  if (g->life != c->life)
    return fail(c, SHAPE_E_INVAL, "the graph was captured on another context");
  if (c->capturing) return fail(c, SHAPE_E_UNSUPPORTED, "graph launch during capture");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, hipGraphLaunch(g->exec, (hipStream_t)stream), "hipGraphLaunch");
  return SHAPE_OK;
}

void shape_graph_destroy(shape_graph* g) {
  if (!g) return;
  if (g->exec) {
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();  // no replay of it is still queued
    (void)hipGraphExecDestroy(g->exec);
  }
  if (g->life) {
    std::lock_guard<std::mutex> lk(g->life->m);
    if (--g->life->live == 0) {
      // the last graph that could address the retired buffers is gone
      for (void* p : g->life->retired) (void)hipFree(p);
      g->life->retired.clear();
      g->life->retired_bytes = 0;
    }
  }
  delete g;
}

int shape_memory_info(const shape_ctx* c, int64_t* scratch_bytes, int64_t* retired_bytes,
                      int32_t* live_graphs) {
  if (!c) return SHAPE_E_INVAL;
  size_t held = 0;
  for (const auto& b : c->buf) held += b.bytes;
  std::lock_guard<std::mutex> lk(c->life->m);
  if (scratch_bytes) *scratch_bytes = (int64_t)held;
  if (retired_bytes) *retired_bytes = (int64_t)c->life->retired_bytes;
  if (live_graphs) *live_graphs = c->life->live;
  return SHAPE_OK;
}

}  // extern "C"
