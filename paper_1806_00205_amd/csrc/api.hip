// Host runtime behind the C interface of rtmc.h: contexts, scenes, tables,
// the chunked generation-by-generation launch sequence of a trace, HIP graph
// replay for batches, and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rtmc.h"
#include "bvh_build.h"
#include "mlp_kernels.h"
#include "rtmc_internal.h"
#include "shade_kernels.h"

using namespace rtmc;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Scene {
  int64_t n_in = 0, n_tris = 0, dropped = 0;
  double lo[3], hi[3];
  uint32_t flags = 0;
  DevBuf tris_in;  // compacted, caller order (freed after the build)
  DevBuf tris;     // Morton order
  DevBuf tris_t;   // the same as rotated 64-byte records, what traversal reads
  DevBuf nodes;    // binary LBVH (64 B per node)
  DevBuf nodes4;   // quantized 4-wide nodes collapsed from it (64 B per node), what traversal reads
  int64_t n_nodes = 0;
  int built = 0, depth = 0;
  double build_ms = 0.0;
};

struct Surrogate {
  int n_in = 0, width = 256, depth = 4;
  int64_t n_pub = 0, n_pad = 0;  // public and padded (first layer 32 wide) parameter counts
  DevBuf master, mom1, mom2, grad;  // FP32, padded layout
  DevBuf wbf;                       // BF16 weights: W_l and W_l^T per layer
  int64_t step = 0;
  // training: per-workgroup bias and loss slices, pre-activations, transposed tiles, loss word
  DevBuf tws;
  int tws_grid = 0;
  // device training loop: state words, learning rates, losses
  DevBuf tbuf;
  hipGraphExec_t tgexec = nullptr;  // one loop step, captured
  std::vector<uint64_t> tkey;       // what that capture depends on
};

struct Tables {
  DevBuf buf;  // yield | cdf_E | cdf_F | esee (paper emission) | guide F | guide E (uint16)
  int32_t nE = 0, nth = 0, ncdf = 0, emission = 0;
  uint32_t e1bits = 0, eshift = 0;
  double Emin = 0, Emax = 0, Ec = 0;
  int max_d = 1;
};

}  // namespace

// ---- scratch memory of the entry points that allocate nothing
//
// One array per GPU, in the library's code object: rtmc_first_hit_noalloc
// keeps its traversal scratch (work counter, error word, job record, hit
// record streams, global traversal stack) here instead of allocating it.
// In host code `scratch` only names the symbol; its device address on each
// GPU is looked up once (rtmc_create) and kept in scratch_dev[].
namespace {
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int64_t kNoAllocMaxRays = (int64_t)1 << 19;
constexpr size_t kScratchHead = 4096;  // work counter, error word, job record (at byte 256)
constexpr size_t kScratchStack = kScratchBytes - kScratchHead - 20 * (size_t)kNoAllocMaxRays;
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static_assert(256 + sizeof(rtmc::DevJob) <= kScratchHead, "job record must fit the scratch head");

// One job record written by the device, so that no host staging buffer is needed.
__global__ void k_store_job(rtmc::DevJob* dst, rtmc::DevJob v) { *dst = v; }

namespace {
hipError_t launch_store_job(rtmc::DevJob* dst, const rtmc::DevJob& v, hipStream_t s) {
  k_store_job<<<1, 1, 0, s>>>(dst, v);
  return hipGetLastError();
}

// Device address of this GPU's scratch array (the device must be current).
hipError_t resolve_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_dev[device] = p;
  }
  *out = scratch_dev[device];
  return hipSuccess;
}
}  // namespace

struct rtmc_ctx {
  int device = 0;
  void* scratch = nullptr;  // this device's scratch array (rtmc_first_hit_noalloc)
  hipStream_t stream = nullptr;
  hipStream_t gstream = nullptr;  // graph capture / replay
  rtmc_allocator alloc{};
  bool custom_alloc = false;
  std::string err;
  int n_cu = 0;
  size_t lds_per_block = 0;
  std::vector<Scene> scenes;
  std::vector<Tables> tables;
  std::vector<Surrogate> srgs;
  rtmc_launch_cfg cfg{256, 7, 16, 1 << 24, 48, 0, kClaimDefault};
  // trace work buffers, grown on demand
  DevBuf queue[2];
  DevBuf hits;  // hit records, qcap entries
  uint32_t qcap = 0;
  DevBuf gstack;
  DevBuf counters, ppc, err_word, jobs, tally;
  // pinned host copy of the error word and the tallies: read back with
  // asynchronous copies queued behind the kernels, one synchronization per trace
  void* pin = nullptr;
  size_t pin_bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<hipEvent_t> kev;  // per-launch timing events (eager traces)
  // replay output requested by the current rtmc_trace (queued rays of one generation)
  float* replay = nullptr;
  uint32_t n_replay = 0;
  int32_t replay_gen = 0;
  // last instantiated batch graph and the signature it was captured for
  hipGraphExec_t gexec = nullptr;
  std::vector<uint64_t> gkey;
};

namespace {

rtmc_status fail(rtmc_ctx* c, rtmc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

#define HIPCHK(c, expr)                                                                                 \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess) return fail((c), RTMC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

void* dev_alloc(rtmc_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (c->custom_alloc) return c->alloc.alloc(bytes, c->alloc.user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dev_free(rtmc_ctx* c, DevBuf& b) {
  if (!b.p) return;
  if (c->custom_alloc)
    c->alloc.free(b.p, c->alloc.user);
  else
    (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

rtmc_status ensure(rtmc_ctx* c, DevBuf& b, size_t bytes) {
  if (b.p && b.bytes >= bytes) return RTMC_OK;
  dev_free(c, b);
  b.p = dev_alloc(c, bytes);
  if (!b.p) return fail(c, RTMC_ENOMEM, "device allocation of %zu bytes failed", bytes);
  b.bytes = bytes;
  return RTMC_OK;
}

rtmc_status check_scene(rtmc_ctx* c, int32_t id, bool need_bvh) {
  if (!c) return RTMC_EINVAL;
  if (id < 0 || id >= (int32_t)c->scenes.size()) return fail(c, RTMC_EINVAL, "unknown scene id %d", id);
  if (need_bvh && !c->scenes[id].built) return fail(c, RTMC_ESTATE, "scene %d has no BVH: call rtmc_build_bvh", id);
  return RTMC_OK;
}

// Queue the copies of the error word and n_words tally words into the pinned
// host buffer (grown when needed; no copy is in flight when this is called).
hipError_t queue_readback(rtmc_ctx* c, size_t n_words, hipStream_t s) {
  const size_t need = 16 + n_words * 8;
  if (c->pin_bytes < need) {
    if (c->pin) (void)hipHostFree(c->pin);
    c->pin = nullptr;
    c->pin_bytes = 0;
    hipError_t e = hipHostMalloc(&c->pin, need, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    c->pin_bytes = need;
  }
  hipError_t e = hipMemcpyAsync(c->pin, c->err_word.p, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && n_words)
    e = hipMemcpyAsync(static_cast<char*>(c->pin) + 16, c->tally.p, n_words * 8, hipMemcpyDeviceToHost, s);
  return e;
}

DevScene dev_scene(const Scene& s) {
  DevScene d;
  d.nodes = reinterpret_cast<const float4*>(s.nodes4.p);
  d.tris = reinterpret_cast<const float4*>(s.tris.p);
  d.tris_t = reinterpret_cast<const float4*>(s.tris_t.p);
  double w = 0.0;
  for (int a = 0; a < 3; ++a) {
    d.lo[a] = (float)s.lo[a];
    d.hi[a] = (float)s.hi[a];
    w = std::max(w, std::max(std::fabs(s.lo[a]), std::fabs(s.hi[a])));
  }
  // every vertex lies in the box; a quantized node plane overshoots the
  // bound by less than one code step, at most 4/255 of it
  d.wext = (float)(w * 1.03);
  d.n_tris = (int32_t)s.n_tris;
  d.flags = s.flags;
  return d;
}

DevTables dev_tables(const Tables& t) {
  DevTables d;
  const float* base = reinterpret_cast<const float*>(t.buf.p);
  d.yld = base;
  d.cdfE = base + (size_t)t.nE * t.nth;
  d.cdfF = d.cdfE + t.ncdf;
  d.nE = t.nE;
  d.nth = t.nth;
  d.ncdf = t.ncdf;
  d.logEmin = (float)std::log(t.Emin);
  d.invdlogE = (float)((t.nE - 1) / (std::log(t.Emax) - std::log(t.Emin)));
  d.thscale = (float)((t.nth - 1) / 90.0);
  d.Ec = (float)t.Ec;
  d.esee = t.emission == RTMC_EMIT_PAPER ? d.cdfF + t.ncdf : nullptr;
  d.emission = t.emission;
  const float* gbase = d.cdfF + t.ncdf + (t.emission == RTMC_EMIT_PAPER ? (size_t)t.nE * t.nth : 0);
  d.gF = reinterpret_cast<const uint16_t*>(gbase);
  d.gE = d.gF + kGuide;
  d.e1bits = t.e1bits;
  d.eshift = t.eshift;
  return d;
}

int grid_of(const rtmc_ctx* c, const rtmc_launch_cfg& cfg) { return c->n_cu * cfg.wg_per_cu; }

// Traversal stack entries a ray can need in a BVH of `depth` binary levels:
// each 4-wide node descends at least one level and pushes at most three children.
int stack_need(int depth) { return 3 * depth + 2; }

struct HostJob {
  int32_t scene;
  double E, theta;
  uint64_t n, seed, pid0;
  uint32_t* pp;
};

struct TraceOut {
  std::vector<unsigned long long> tally;  // n_jobs blocks
  int n_chunks = 0;
  double ms = 0.0;
  double kernel_ms = 0.0;
  double shade_ms = 0.0;
  uint64_t launches = 0;
};

HitRecs hit_recs(void* base, size_t cap) {
  HitRecs h;
  uint32_t* u = reinterpret_cast<uint32_t*>(base);
  h.code = reinterpret_cast<int32_t*>(u);
  h.f0 = reinterpret_cast<float*>(u + cap);
  h.f1 = reinterpret_cast<float*>(u + 2 * cap);
  h.t = reinterpret_cast<float*>(u + 3 * cap);
  h.visits = u + 4 * cap;
  h.tests = u + 5 * cap;
  h.wraps = u + 6 * cap;
  return h;
}

constexpr int kShadeBlock = 1024;  // k_shade workgroup: 16 waves share one queue reservation per step

// One chunk of the batch: primaries [lo, lo + n) of the concatenated jobs,
// which lie in jobs j_lo..j_hi.
struct ChunkPlan {
  uint64_t lo;
  uint32_t n;
  int32_t j_lo, j_hi;
};

// Cut the concatenated primaries into chunks of at most `chunk`.  A chunk is
// also closed before it would span more than kShadeJobs jobs, once it holds a
// quarter of `chunk`: shading then keeps every job's tallies in LDS, while
// batches of many small jobs still get chunks large enough to fill the device.
std::vector<ChunkPlan> plan_chunks(const std::vector<HostJob>& jobs, uint32_t chunk) {
  std::vector<ChunkPlan> out;
  ChunkPlan cur{0, 0, -1, -1};
  uint64_t g = 0;
  const uint32_t min_fill = std::max<uint32_t>(1u, chunk / 4);
  for (int32_t j = 0; j < (int32_t)jobs.size(); ++j) {
    uint64_t left = jobs[j].n;
    while (left > 0) {
      if (cur.n > 0 && (cur.n == chunk || (j - cur.j_lo + 1 > kShadeJobs && cur.n >= min_fill))) {
        out.push_back(cur);
        cur = ChunkPlan{g, 0, -1, -1};
      }
      if (cur.n == 0) {
        cur.lo = g;
        cur.j_lo = j;
      }
      const uint32_t take = (uint32_t)std::min<uint64_t>(left, (uint64_t)(chunk - cur.n));
      cur.n += take;
      cur.j_hi = j;
      left -= take;
      g += take;
    }
  }
  if (cur.n > 0) out.push_back(cur);
  return out;
}

// Rays of several scenes in one launch: traversal then takes each ray's scene
// from its job (the batched kernel); jobs that share one scene use the
// single-scene kernel.
bool multi_scene(const std::vector<HostJob>& jobs) {
  for (auto& j : jobs)
    if (j.scene != jobs[0].scene) return true;
  return false;
}

// Enqueue the launch sequence of a batch of jobs with a given chunk size:
// per chunk and generation, traversal then shading.
rtmc_status enqueue_trace(rtmc_ctx* c, const Tables& tb, const std::vector<HostJob>& jobs, int max_gen,
                          int n_ebins, int n_abins, int n_zbins, const rtmc_launch_cfg& cfg, uint32_t chunk,
                          hipStream_t s,
                          uint64_t total, bool timed, uint64_t* n_launch) {
  const int block = cfg.block;
  const int grid = grid_of(c, cfg);
  const std::vector<ChunkPlan> plan = plan_chunks(jobs, chunk);
  const uint64_t n_chunks = plan.size();
  (void)total;
  const size_t tw = (size_t)T_NCOUNT + n_ebins + n_abins + n_zbins;
  const int ncnt = 2 * (kMaxGen + 2);
  int gdepth = kGlobalStack;
  for (auto& j : jobs) gdepth = std::max(gdepth, stack_need(c->scenes[j.scene].depth));
  const bool multi = multi_scene(jobs);

  HIPCHK(c, launch_fill_u64(reinterpret_cast<unsigned long long*>(c->tally.p), 0ull, tw * jobs.size(), s));
  HIPCHK(c, launch_fill_u32(reinterpret_cast<uint32_t*>(c->counters.p), 0u, (size_t)ncnt * n_chunks, s));
  HIPCHK(c, launch_fill_u32(reinterpret_cast<uint32_t*>(c->err_word.p), 0u, 2, s));

  // the whole allocated queue is the limit: after an overflow the chunk is
  // halved while the queue keeps its length, so every retry doubles the
  // room per primary
  const uint32_t qcap = c->qcap;
  (void)chunk;
  RayQueue q[2];
  for (int i = 0; i < 2; ++i) {
    float* f = reinterpret_cast<float*>(c->queue[i].p);
    const size_t Q = c->qcap;
    q[i].ox = f;
    q[i].oy = f + Q;
    q[i].oz = f + 2 * Q;
    q[i].dx = f + 3 * Q;
    q[i].dy = f + 4 * Q;
    q[i].dz = f + 5 * Q;
    q[i].E = f + 6 * Q;
    q[i].path = reinterpret_cast<uint32_t*>(f + 7 * Q);
    q[i].ci = reinterpret_cast<uint32_t*>(f + 8 * Q);
    q[i].meta = reinterpret_cast<uint32_t*>(f + 9 * Q);
  }
  const HitRecs hr = hit_recs(c->hits.p, c->qcap);
  uint32_t* errw = reinterpret_cast<uint32_t*>(c->err_word.p);

  TraverseArgs ta{};
  ta.jobs = reinterpret_cast<const DevJob*>(c->jobs.p);
  ta.n_jobs = (int32_t)jobs.size();
  ta.qcap = qcap;
  ta.hit = hr;
  ta.gstack = reinterpret_cast<uint32_t*>(c->gstack.p);
  ta.lds_stack = cfg.lds_stack;
  ta.gstack_depth = gdepth;
  ta.refill = cfg.refill;
  ta.claim_max = (uint32_t)cfg.claim;
  ta.err = errw;

  ShadeArgs sa{};
  sa.jobs = ta.jobs;
  sa.n_jobs = ta.n_jobs;
  sa.tb = dev_tables(tb);
  sa.qcap = qcap;
  sa.ppc = reinterpret_cast<uint32_t*>(c->ppc.p);
  sa.max_gen = max_gen;
  sa.n_ebins = n_ebins;
  sa.n_abins = n_abins;
  sa.n_zbins = n_zbins;
  sa.hit = hr;
  sa.err = errw;

  auto ev = [&](size_t k) -> hipEvent_t {
    while (c->kev.size() <= k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      c->kev.push_back(e);
    }
    return c->kev[k];
  };
  for (uint64_t ch = 0; ch < n_chunks; ++ch) {
    const uint64_t lo = plan[ch].lo;
    const uint32_t n_here = plan[ch].n;
    uint32_t* cnt = reinterpret_cast<uint32_t*>(c->counters.p) + ch * ncnt;
    const int32_t j_lo = plan[ch].j_lo, j_hi = plan[ch].j_hi;
    HIPCHK(c, launch_fill_u32(sa.ppc, 0u, n_here, s));
    HIPCHK(c, launch_primaries(ta.jobs, j_lo, j_hi, lo, n_here, q[0], s));
    sa.j_lo = j_lo;
    sa.j_hi = j_hi;
    ta.chunk_lo = sa.chunk_lo = lo;
    sa.n_gen0 = n_here;
    for (int g = 0; g <= max_gen; ++g) {
      ta.src = 1;
      ta.count = n_here;
      ta.qin = q[g & 1];
      ta.count_in = g == 0 ? nullptr : cnt + g;  // produced by generation g - 1
      ta.work = cnt + (kMaxGen + 2) + g;
      sa.gen = g;
      sa.qin = q[g & 1];
      sa.qout = q[(g + 1) & 1];
      sa.count_in = cnt + g;
      sa.count_out = cnt + g + 1;
      if (timed) {
        // three events per generation: before traversal, between the launches, after shading
        const size_t k = 3 * (size_t)(*n_launch);
        hipEvent_t e0 = ev(k), e1 = ev(k + 1), e2 = ev(k + 2);
        if (!e0 || !e1 || !e2) return fail(c, RTMC_EDEVICE, "event creation failed");
        HIPCHK(c, hipEventRecord(e0, s));
        HIPCHK(c, launch_traverse(ta, multi, cfg.occupancy, grid, block, s));
        HIPCHK(c, hipEventRecord(e1, s));
        HIPCHK(c, launch_shade(sa, c->n_cu, kShadeBlock, s));
        HIPCHK(c, hipEventRecord(e2, s));
      } else {
        HIPCHK(c, launch_traverse(ta, multi, cfg.occupancy, grid, block, s));
        HIPCHK(c, launch_shade(sa, c->n_cu, kShadeBlock, s));
      }
      ++*n_launch;
      if (ch == 0 && c->replay && g + 1 == c->replay_gen)
        HIPCHK(c, launch_copy_rays(q[(g + 1) & 1], cnt + g + 1, qcap, c->replay, c->n_replay, errw + 1, s));
    }
    HIPCHK(c, launch_chunk_reduce(ta.jobs, j_lo, j_hi, sa.ppc, n_here, lo, s));
  }
  return RTMC_OK;
}

rtmc_status prepare_trace(rtmc_ctx* c, const Tables& tb, const std::vector<HostJob>& jobs, int n_ebins, int n_abins,
                          int n_zbins,
                          const rtmc_launch_cfg& cfg, uint64_t* total_out) {
  // job table
  std::vector<DevJob> dj(jobs.size());
  const size_t tw = (size_t)T_NCOUNT + n_ebins + n_abins + n_zbins;
  rtmc_status st = ensure(c, c->tally, tw * jobs.size() * 8);
  if (st) return st;
  uint64_t g = 0;
  for (size_t i = 0; i < jobs.size(); ++i) {
    const Scene& sc = c->scenes[jobs[i].scene];
    dj[i].sc = dev_scene(sc);
    dj[i].E0 = (float)jobs[i].E;
    dj[i].theta = (float)jobs[i].theta;
    dj[i].seed = jobs[i].seed;
    dj[i].pid0 = jobs[i].pid0;
    dj[i].n_prim = jobs[i].n;
    dj[i].gbase = g;
    dj[i].tally = reinterpret_cast<unsigned long long*>(c->tally.p) + tw * i;
    dj[i].pp_escaped = jobs[i].pp;
    g += jobs[i].n;
  }
  *total_out = g;
  st = ensure(c, c->jobs, sizeof(DevJob) * dj.size());
  if (st) return st;
  HIPCHK(c, hipMemcpyAsync(c->jobs.p, dj.data(), sizeof(DevJob) * dj.size(), hipMemcpyHostToDevice, c->stream));
  const uint32_t chunk = (uint32_t)cfg.chunk;
  // queues sized for the largest chunk this trace plans (at most `chunk` primaries)
  uint64_t max_chunk = 1;
  for (const ChunkPlan& p : plan_chunks(jobs, chunk)) max_chunk = std::max<uint64_t>(max_chunk, p.n);
  const uint64_t need_q = max_chunk * tb.max_d;
  // the 32-bit work counters may run past the queue length by one block claim per wave
  const uint64_t claim_slack = (uint64_t)grid_of(c, cfg) * (cfg.block / 64) * (uint64_t)cfg.claim;
  if (need_q + claim_slack > 0xFFFFFFF0ull) return fail(c, RTMC_EINVAL, "chunk too large for the queue index range");
  if (c->qcap < need_q || !c->queue[0].p) {
    for (int i = 0; i < 2; ++i) {
      st = ensure(c, c->queue[i], (size_t)need_q * 40);
      if (st) return st;
    }
    st = ensure(c, c->hits, (size_t)need_q * 28);
    if (st) return st;
    c->qcap = (uint32_t)need_q;
  }
  const uint64_t n_chunks = plan_chunks(jobs, chunk).size();
  st = ensure(c, c->counters, (size_t)n_chunks * 2 * (kMaxGen + 2) * 4 + 16);
  if (st) return st;
  st = ensure(c, c->ppc, (size_t)chunk * 4);
  if (st) return st;
  st = ensure(c, c->err_word, 16);
  if (st) return st;
  int gdepth = kGlobalStack;
  for (auto& j : jobs) gdepth = std::max(gdepth, stack_need(c->scenes[j.scene].depth));
  const size_t waves = (size_t)grid_of(c, cfg) * (cfg.block / 64);
  st = ensure(c, c->gstack, waves * gdepth * 64 * 4);
  if (st) return st;
  return RTMC_OK;
}

rtmc_status run_trace(rtmc_ctx* c, int32_t table_id, std::vector<HostJob>& jobs, int max_gen, int n_ebins,
                      int n_abins, int n_zbins, bool use_graph, TraceOut& out) {
  const Tables& tb = c->tables[table_id];
  rtmc_launch_cfg cfg = c->cfg;
  const size_t tw = (size_t)T_NCOUNT + n_ebins + n_abins + n_zbins;
  for (int attempt = 0;; ++attempt) {
    uint64_t total = 0;
    rtmc_status st = prepare_trace(c, tb, jobs, n_ebins, n_abins, n_zbins, cfg, &total);
    if (st) return st;
    const size_t lds_t = traverse_lds_bytes(cfg.lds_stack, cfg.block);
    // shading keeps per-job tallies in LDS for chunks of at most kShadeJobs jobs
    int max_jobs = 1;
    for (const ChunkPlan& p : plan_chunks(jobs, (uint32_t)cfg.chunk)) max_jobs = std::max(max_jobs, p.j_hi - p.j_lo + 1);
    const size_t lds_s = shade_lds_bytes(dev_tables(tb), n_ebins + n_abins + n_zbins, kShadeBlock, max_jobs);
    if (lds_t > c->lds_per_block || lds_s > c->lds_per_block)
      return fail(c, RTMC_EINVAL, "launch needs %zu / %zu bytes of LDS per workgroup (device limit %zu)", lds_t,
                  lds_s, c->lds_per_block);
    hipStream_t s = use_graph ? c->gstream : c->stream;
    if (use_graph) {
      HIPCHK(c, hipEventRecord(c->ev0, c->stream));
      HIPCHK(c, hipStreamWaitEvent(c->gstream, c->ev0, 0));
      // The graph depends on the launch sequence (sizes, shapes) and on the
      // device buffers it names, not on the job table's contents, which are
      // uploaded to the same buffer before every launch.
      std::vector<uint64_t> key = {(uint64_t)jobs.size(), total, (uint64_t)max_gen, (uint64_t)n_ebins,
                                   (uint64_t)n_abins, (uint64_t)n_zbins, (uint64_t)cfg.block,
                                   (uint64_t)cfg.wg_per_cu,
                                   (uint64_t)cfg.lds_stack, (uint64_t)cfg.chunk, (uint64_t)cfg.refill,
                                   (uint64_t)cfg.occupancy, (uint64_t)cfg.claim, (uint64_t)table_id,
                                   (uint64_t)(uintptr_t)c->jobs.p,
                                   (uint64_t)(uintptr_t)c->tally.p, (uint64_t)(uintptr_t)c->queue[0].p,
                                   (uint64_t)(uintptr_t)c->queue[1].p, (uint64_t)(uintptr_t)c->hits.p,
                                   (uint64_t)(uintptr_t)c->counters.p, (uint64_t)(uintptr_t)c->ppc.p,
                                   (uint64_t)(uintptr_t)c->gstack.p, (uint64_t)(uintptr_t)c->err_word.p, c->qcap};
      int gd = kGlobalStack;
      for (auto& j : jobs) gd = std::max(gd, stack_need(c->scenes[j.scene].depth));
      key.push_back((uint64_t)gd);
      key.push_back(multi_scene(jobs) ? 1u : 0u);
      // the per-job primary counts fix each chunk's job range, baked into the launches
      for (auto& j : jobs) key.push_back(j.n);
      uint64_t nl = 0;
      if (!c->gexec || key != c->gkey) {
        if (c->gexec) {
          (void)hipGraphExecDestroy(c->gexec);
          c->gexec = nullptr;
        }
        hipGraph_t graph = nullptr;
        HIPCHK(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        st = enqueue_trace(c, tb, jobs, max_gen, n_ebins, n_abins, n_zbins, cfg, (uint32_t)cfg.chunk, s, total,
                           false, &nl);
        hipError_t ce = hipStreamEndCapture(s, &graph);
        if (st) {
          if (graph) (void)hipGraphDestroy(graph);
          return st;
        }
        HIPCHK(c, ce);
        hipError_t ie = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(c, ie);
        c->gkey = key;
      } else {
        nl = (uint64_t)plan_chunks(jobs, (uint32_t)cfg.chunk).size() * (uint64_t)(max_gen + 1);
      }
      out.launches = nl;
      out.kernel_ms = 0.0;
      HIPCHK(c, hipEventRecord(c->ev0, s));
      hipError_t le = hipGraphLaunch(c->gexec, s);
      HIPCHK(c, hipEventRecord(c->ev1, s));
      HIPCHK(c, queue_readback(c, tw * jobs.size(), s));
      hipError_t se = hipStreamSynchronize(s);
      HIPCHK(c, le);
      HIPCHK(c, se);
    } else {
      HIPCHK(c, hipEventRecord(c->ev0, s));
      uint64_t nl = 0;
      st = enqueue_trace(c, tb, jobs, max_gen, n_ebins, n_abins, n_zbins, cfg, (uint32_t)cfg.chunk, s, total, true,
                         &nl);
      if (st) return st;
      HIPCHK(c, hipEventRecord(c->ev1, s));
      HIPCHK(c, queue_readback(c, tw * jobs.size(), s));
      HIPCHK(c, hipStreamSynchronize(s));
      double kms = 0.0, sms = 0.0;
      for (uint64_t i = 0; i < nl; ++i) {
        float e = 0.f;
        HIPCHK(c, hipEventElapsedTime(&e, c->kev[3 * i], c->kev[3 * i + 1]));
        kms += e;
        HIPCHK(c, hipEventElapsedTime(&e, c->kev[3 * i + 1], c->kev[3 * i + 2]));
        sms += e;
      }
      out.kernel_ms = kms;
      out.shade_ms = sms;
      out.launches = nl;
    }
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    uint32_t errw = 0;
    std::memcpy(&errw, c->pin, 4);
    if (errw & 2u) return fail(c, RTMC_EOVERFLOW, "traversal stack overflow (BVH deeper than the stack)");
    if (errw & 1u) {
      // a generation outgrew the queue: trace again with chunks half the size
      // of the largest one just planned (the queue keeps its length)
      uint32_t largest = 1;
      for (const ChunkPlan& p : plan_chunks(jobs, (uint32_t)cfg.chunk)) largest = std::max(largest, p.n);
      if (largest <= 1)
        return fail(c, RTMC_EOVERFLOW, "one primary's ray tree does not fit the daughter queue");
      cfg.chunk = (int32_t)(largest / 2);
      continue;
    }
    out.tally.resize(tw * jobs.size());
    std::memcpy(out.tally.data(), static_cast<const char*>(c->pin) + 16, out.tally.size() * 8);
    out.ms = ms;
    out.n_chunks = (int)plan_chunks(jobs, (uint32_t)cfg.chunk).size();
    (void)attempt;
    return RTMC_OK;
  }
}

void fill_result(const unsigned long long* t, const HostJob& j, int n_ebins, int n_abins, int n_zbins, uint64_t* eh,
                 uint64_t* ah, uint64_t* zh, const TraceOut& to, rtmc_result* r) {
  std::memset(r, 0, sizeof(*r));
  r->n_primaries = j.n;
  r->n_rays = t[T_RAYS];
  r->n_escaped = t[T_ESCAPED];
  r->n_absorbed = t[T_ABSORBED];
  r->n_truncated = t[T_TRUNCATED];
  r->n_lost = t[T_LOST];
  r->n_substrate = t[T_SUBSTRATE];
  r->n_wraps = t[T_WRAPS];
  r->n_node_visits = t[T_VISITS];
  r->n_tri_tests = t[T_TESTS];
  r->n_spawned = t[T_SPAWNED];
  r->e_escaped = (double)(long long)t[T_E_ESC_FX] / kFixScale;
  r->e_deposited = (double)(long long)t[T_E_DEP_FX] / kFixScale;
  const double N = (double)j.n;
  if (N > 0) {
    const double mean = (double)t[T_ESCAPED] / N;
    r->yield = mean;
    double var = N > 1 ? ((double)t[T_C2] - N * mean * mean) / (N - 1.0) : 0.0;
    if (var < 0) var = 0;
    r->yield_sigma = std::sqrt(var / N);
  }
  r->ms = to.ms;
  r->kernel_ms = to.kernel_ms;
  r->shade_ms = to.shade_ms;
  r->n_kernel_launches = to.launches;
  r->n_chunks = to.n_chunks;
  if (eh)
    for (int b = 0; b < n_ebins; ++b) eh[b] = t[T_NCOUNT + b];
  if (ah)
    for (int b = 0; b < n_abins; ++b) ah[b] = t[T_NCOUNT + n_ebins + b];
  if (zh)
    for (int b = 0; b < n_zbins; ++b) zh[b] = t[T_NCOUNT + n_ebins + n_abins + b];
}

bool finite_f(float x) { return std::isfinite(x); }

// A batch whose sequence holds more traversal launches than this is replayed as a HIP graph.
constexpr uint64_t kGraphLaunches = 128;

// Launch shapes chosen by rtmc_autotune, for the process: the GPU, the
// scene's size class, the tables' largest yield and the calibration point.
using TuneKey = std::vector<uint64_t>;
std::mutex tune_mu;
std::vector<std::pair<TuneKey, rtmc_launch_cfg>> tune_cache;

TuneKey tune_key(const rtmc_ctx* c, int32_t scene_id, int32_t table_id, double E, double theta, uint64_t n) {
  const Scene& s = c->scenes[scene_id];
  hipDeviceProp_t prop;
  uint64_t arch = 0;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess)
    for (const char* p = prop.gcnArchName; *p; ++p) arch = arch * 131 + (unsigned char)*p;
  uint64_t tri_bucket = 0;
  while ((1ull << tri_bucket) < (uint64_t)std::max<int64_t>(s.n_tris, 1)) ++tri_bucket;
  uint64_t eb, tb;
  std::memcpy(&eb, &E, 8);
  std::memcpy(&tb, &theta, 8);
  return {arch, (uint64_t)c->n_cu, tri_bucket, (uint64_t)s.depth, (uint64_t)c->tables[table_id].max_d,
          (uint64_t)s.flags, eb, tb, n};
}

}  // namespace

extern "C" {

rtmc_status rtmc_create(rtmc_ctx** out, int device, const rtmc_allocator* alloc, void* hip_stream) {
  if (!out) return RTMC_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return RTMC_EDEVICE;
  if (device < 0 || device >= ndev) return RTMC_EINVAL;
  if (alloc && (!alloc->alloc || !alloc->free)) return RTMC_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return RTMC_EDEVICE;
  rtmc_ctx* c = new rtmc_ctx();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (alloc) {
    c->alloc = *alloc;
    c->custom_alloc = true;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess || hipStreamCreate(&c->gstream) != hipSuccess ||
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    rtmc_destroy(c);
    return RTMC_EDEVICE;
  }
  c->n_cu = prop.multiProcessorCount;
  c->lds_per_block = prop.sharedMemPerBlock;
  if (resolve_scratch(device, &c->scratch) != hipSuccess) {
    rtmc_destroy(c);
    return RTMC_EDEVICE;
  }
  *out = c;
  return RTMC_OK;
}

void rtmc_destroy(rtmc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->gstream) (void)hipStreamSynchronize(c->gstream);
  for (auto& s : c->scenes) {
    dev_free(c, s.tris_in);
    dev_free(c, s.tris);
    dev_free(c, s.tris_t);
    dev_free(c, s.nodes);
    dev_free(c, s.nodes4);
  }
  for (auto& t : c->tables) dev_free(c, t.buf);
  for (auto& g : c->srgs) {
    if (g.tgexec) (void)hipGraphExecDestroy(g.tgexec);
    dev_free(c, g.tbuf);
    dev_free(c, g.master);
    dev_free(c, g.mom1);
    dev_free(c, g.mom2);
    dev_free(c, g.grad);
    dev_free(c, g.wbf);
    dev_free(c, g.tws);
  }
  dev_free(c, c->queue[0]);
  dev_free(c, c->queue[1]);
  dev_free(c, c->hits);
  dev_free(c, c->gstack);
  dev_free(c, c->counters);
  dev_free(c, c->ppc);
  dev_free(c, c->err_word);
  dev_free(c, c->jobs);
  dev_free(c, c->tally);
  if (c->pin) (void)hipHostFree(c->pin);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  for (auto e : c->kev) (void)hipEventDestroy(e);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  delete c;
}

const char* rtmc_last_error(const rtmc_ctx* c) { return c ? c->err.c_str() : "null context"; }

rtmc_status rtmc_set_stream(rtmc_ctx* c, void* hip_stream) {
  if (!c) return RTMC_EINVAL;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return RTMC_OK;
}

namespace {
rtmc_status load_mesh_impl(rtmc_ctx* c, const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                           const double box_lo[3], const double box_hi[3], uint32_t flags, int32_t* scene_id) {
  c->err.clear();
  if (!scene_id || !box_lo || !box_hi || n_verts < 0 || n_tris < 0 || (n_verts > 0 && !verts) ||
      (n_tris > 0 && !tris))
    return fail(c, RTMC_EINVAL, "null pointer or negative size");
  if (n_tris >= (int64_t)0x7fffffff) return fail(c, RTMC_EINVAL, "too many triangles (%lld)", (long long)n_tris);
  if (flags & ~(RTMC_PERIODIC_XY | RTMC_SUBSTRATE)) return fail(c, RTMC_EINVAL, "unknown flag bits");
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(box_lo[a]) || !std::isfinite(box_hi[a]) || !(box_hi[a] > box_lo[a]))
      return fail(c, RTMC_EINVAL, "box axis %d is empty or not finite", a);
  }
  // validation and packing run over host threads in contiguous ranges; the
  // first offending vertex or triangle in index order is the one reported
  const int nth = n_verts + n_tris < (1 << 16) ? 1 : (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto ranges = [nth](int64_t n, auto&& f) {
    std::vector<std::thread> ts;
    for (int t = 0; t < nth; ++t) {
      const int64_t lo = n * t / nth, hi = n * (t + 1) / nth;
      if (t + 1 < nth)
        ts.emplace_back(f, t, lo, hi);
      else
        f(t, lo, hi);
    }
    for (auto& th : ts) th.join();
  };
  // vertices: the first non-finite or out-of-box coordinate
  std::vector<int64_t> bad_v(nth, -1);
  std::vector<int> bad_v_kind(nth, 0);
  ranges(n_verts, [&](int t, int64_t lo, int64_t hi) {
    for (int64_t v = lo; v < hi; ++v)
      for (int a = 0; a < 3; ++a) {
        const float x = verts[3 * v + a];
        const int kind = !finite_f(x) ? 1 : ((double)x < box_lo[a] || (double)x > box_hi[a]) ? 2 : 0;
        if (kind) {
          bad_v[t] = v;
          bad_v_kind[t] = kind;
          return;
        }
      }
  });
  for (int t = 0; t < nth; ++t)
    if (bad_v[t] >= 0)
      return fail(c, RTMC_EINVAL, bad_v_kind[t] == 1 ? "vertex %lld is not finite" : "vertex %lld lies outside the box",
                  (long long)bad_v[t]);
  Scene s;
  s.n_in = n_tris;
  std::memcpy(s.lo, box_lo, sizeof(s.lo));
  std::memcpy(s.hi, box_hi, sizeof(s.hi));
  s.flags = flags;
  // triangles, first pass: index range, zero area (dropped: the FP64 cross
  // product of the edges is exactly zero), a surface lying in a face of the
  // cell (refused: it would be met exactly where a ray leaves the cell --
  // re-entry, substrate, escape -- and which comes first would be decided by
  // rounding); kept[j] marks the triangles that go on
  std::unique_ptr<uint8_t[]> kept(new uint8_t[(size_t)std::max<int64_t>(n_tris, 1)]);
  std::vector<int64_t> n_kept(nth, 0), bad_t(nth, -1);
  std::vector<int> bad_t_kind(nth, 0), bad_t_arg(nth, 0);
  ranges(n_tris, [&](int th, int64_t lo, int64_t hi) {
    for (int64_t j = lo; j < hi; ++j) {
      const int32_t* t = tris + 3 * j;
      for (int k = 0; k < 3; ++k)
        if (t[k] < 0 || t[k] >= n_verts) {
          bad_t[th] = j;
          bad_t_kind[th] = 1;
          bad_t_arg[th] = t[k];
          return;
        }
      double v[3][3];
      for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) v[k][a] = verts[3 * (int64_t)t[k] + a];
      const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
      const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
      const double nx = e1[1] * e2[2] - e1[2] * e2[1];
      const double ny = e1[2] * e2[0] - e1[0] * e2[2];
      const double nz = e1[0] * e2[1] - e1[1] * e2[0];
      if (nx == 0.0 && ny == 0.0 && nz == 0.0) {
        kept[j] = 0;
        continue;
      }
      for (int a = 0; a < 3; ++a) {
        const bool on_lo = v[0][a] == box_lo[a] && v[1][a] == box_lo[a] && v[2][a] == box_lo[a];
        const bool on_hi = v[0][a] == box_hi[a] && v[1][a] == box_hi[a] && v[2][a] == box_hi[a];
        if (on_lo || on_hi) {
          bad_t[th] = j;
          bad_t_kind[th] = on_lo ? 2 : 3;
          bad_t_arg[th] = a;
          return;
        }
      }
      kept[j] = 1;
      ++n_kept[th];
    }
  });
  for (int t = 0; t < nth; ++t) {
    if (bad_t[t] < 0) continue;
    if (bad_t_kind[t] == 1)
      return fail(c, RTMC_EINVAL, "triangle %lld has vertex index %d out of range", (long long)bad_t[t], bad_t_arg[t]);
    return fail(c, RTMC_EINVAL, "triangle %lld lies in the %s face of the cell on axis %d", (long long)bad_t[t],
                bad_t_kind[t] == 2 ? "lower" : "upper", bad_t_arg[t]);
  }
  // second pass: the kept triangles' 48-byte records (V0, V1, V2; V0.w = the
  // caller's index) in index order, each range at its prefix offset
  std::vector<int64_t> off(nth + 1, 0);
  for (int t = 0; t < nth; ++t) off[t + 1] = off[t] + n_kept[t];
  const int64_t n_out = off[nth];
  s.dropped = n_tris - n_out;
  std::unique_ptr<float[]> packed(new float[(size_t)std::max<int64_t>(n_out, 1) * 12]);
  ranges(n_tris, [&](int th, int64_t lo, int64_t hi) {
    float* o = packed.get() + 12 * off[th];
    for (int64_t j = lo; j < hi; ++j) {
      if (!kept[j]) continue;
      const int32_t* t = tris + 3 * j;
      for (int k = 0; k < 3; ++k) {
        o[0] = verts[3 * (int64_t)t[k]];
        o[1] = verts[3 * (int64_t)t[k] + 1];
        o[2] = verts[3 * (int64_t)t[k] + 2];
        float w = 0.0f;
        if (k == 0) {
          const int32_t id = (int32_t)j;
          std::memcpy(&w, &id, 4);
        }
        o[3] = w;
        o += 4;
      }
    }
  });
  s.n_tris = n_out;
  const size_t bytes = (size_t)n_out * 48;
  HIPCHK(c, hipSetDevice(c->device));
  s.tris_in.p = dev_alloc(c, bytes);
  if (!s.tris_in.p) return fail(c, RTMC_ENOMEM, "device allocation for %lld triangles failed", (long long)s.n_tris);
  s.tris_in.bytes = bytes;
  if (n_out > 0) {
    hipError_t e = hipMemcpyAsync(s.tris_in.p, packed.get(), bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      dev_free(c, s.tris_in);
      return fail(c, RTMC_EDEVICE, "mesh upload: %s", hipGetErrorString(e));
    }
  }
  c->scenes.push_back(s);
  *scene_id = (int32_t)c->scenes.size() - 1;
  return RTMC_OK;
}
}  // namespace

rtmc_status rtmc_load_mesh(rtmc_ctx* c, const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                           const double box_lo[3], const double box_hi[3], uint32_t flags, int32_t* scene_id) {
  if (!c) return RTMC_EINVAL;
  try {  // host threads and buffers may fail to start or allocate; nothing is thrown across the C interface
    return load_mesh_impl(c, verts, n_verts, tris, n_tris, box_lo, box_hi, flags, scene_id);
  } catch (const std::exception& e) {
    return fail(c, RTMC_ENOMEM, "mesh ingest: %s", e.what());
  }
}

rtmc_status rtmc_build_bvh(rtmc_ctx* c, int32_t scene_id) {
  rtmc_status st = check_scene(c, scene_id, false);
  if (st) return st;
  c->err.clear();
  Scene& s = c->scenes[scene_id];
  HIPCHK(c, hipSetDevice(c->device));
  const int64_t n = s.n_tris;
  if (s.built) return RTMC_OK;
  if (n == 0) {
    s.built = 1;
    s.n_nodes = 0;
    return RTMC_OK;
  }
  const int64_t nn = std::max<int64_t>(n - 1, 1);
  DevBuf tris, tris_t, nodes, nodes4, nodes4b, lv, keys, vals, keys2, vals2, parent, flags, hist, depth;
  auto cleanup = [&]() {
    dev_free(c, nodes4b);
    dev_free(c, lv);
    dev_free(c, keys);
    dev_free(c, vals);
    dev_free(c, keys2);
    dev_free(c, vals2);
    dev_free(c, parent);
    dev_free(c, flags);
    dev_free(c, hist);
    dev_free(c, depth);
  };
  if (ensure(c, tris, (size_t)n * 48) || ensure(c, tris_t, (size_t)n * 64) || ensure(c, nodes, (size_t)nn * 64) || ensure(c, nodes4, (size_t)nn * 64) ||
      ensure(c, keys, (size_t)n * 8) ||
      ensure(c, vals, (size_t)n * 4) || ensure(c, keys2, (size_t)n * 8) || ensure(c, vals2, (size_t)n * 4) ||
      ensure(c, parent, (size_t)(nn + n) * 4) || ensure(c, flags, (size_t)nn * 4) ||
      ensure(c, hist, radix_hist_words(n) * 4) || ensure(c, depth, 16) || ensure(c, nodes4b, (size_t)nn * 64) ||
      ensure(c, lv, (size_t)std::max(2 * kRelayoutLevels, kRefitLevels) * 4)) {
    cleanup();
    dev_free(c, tris);
    dev_free(c, tris_t);
    dev_free(c, nodes);
    dev_free(c, nodes4);
    return RTMC_ENOMEM;
  }
  BvhBuild b;
  b.tris_in = reinterpret_cast<const float4*>(s.tris_in.p);
  b.tris_out = reinterpret_cast<float4*>(tris.p);
  b.tris_rot = reinterpret_cast<float4*>(tris_t.p);
  b.nodes = reinterpret_cast<float4*>(nodes.p);
  b.nodes4 = reinterpret_cast<float4*>(nodes4.p);
  b.keys = reinterpret_cast<uint64_t*>(keys.p);
  b.vals = reinterpret_cast<uint32_t*>(vals.p);
  b.keys_alt = reinterpret_cast<uint64_t*>(keys2.p);
  b.vals_alt = reinterpret_cast<uint32_t*>(vals2.p);
  b.parent = reinterpret_cast<int32_t*>(parent.p);
  b.flags = reinterpret_cast<uint32_t*>(flags.p);
  b.hist = reinterpret_cast<uint32_t*>(hist.p);
  b.depth = reinterpret_cast<uint32_t*>(depth.p);
  b.level_count = reinterpret_cast<uint32_t*>(lv.p);
  b.n = (int32_t)n;
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = (float)s.lo[a];
    b.hi[a] = (float)s.hi[a];
  }
  hipError_t e = hipEventRecord(c->ev0, c->stream);
  if (e == hipSuccess) e = build_bvh(b, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  uint32_t d = 1;
  if (e == hipSuccess && n > 1) e = hipMemcpy(&d, depth.p, 4, hipMemcpyDeviceToHost);
  // breadth-first copy of the reached 4-wide records (the 4-wide depth is at
  // most the binary one); a tree too deep for the level table keeps the
  // collapsed layout, which traversal reads just as well
  const bool relaid = e == hipSuccess && (int64_t)d + 2 <= kRelayoutLevels;
  if (relaid)
    e = relayout_wide(b.nodes4, reinterpret_cast<float4*>(nodes4b.p), nn, b.vals, b.vals_alt,
                      reinterpret_cast<uint32_t*>(lv.p), (int)d + 1, c->stream);
  if (e == hipSuccess) e = hipEventRecord(c->ev1, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && relaid) std::swap(nodes4, nodes4b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev0, c->ev1);
  cleanup();
  if (e != hipSuccess) {
    dev_free(c, tris);
    dev_free(c, tris_t);
    dev_free(c, nodes);
    dev_free(c, nodes4);
    return fail(c, RTMC_EDEVICE, "BVH build: %s", hipGetErrorString(e));
  }
  dev_free(c, s.tris_in);
  s.tris = tris;
  s.tris_t = tris_t;
  s.nodes = nodes;
  s.nodes4 = nodes4;
  s.n_nodes = nn;
  s.depth = (int)d;
  s.build_ms = ms;
  s.built = 1;
  return RTMC_OK;
}

rtmc_status rtmc_get_scene_info(rtmc_ctx* c, int32_t scene_id, rtmc_scene_info* out) {
  rtmc_status st = check_scene(c, scene_id, false);
  if (st) return st;
  if (!out) return fail(c, RTMC_EINVAL, "null output");
  const Scene& s = c->scenes[scene_id];
  out->n_tris_in = s.n_in;
  out->n_tris = s.n_tris;
  out->n_dropped = s.dropped;
  out->n_nodes = s.n_nodes;
  out->bvh_built = s.built;
  out->bvh_depth = s.depth;
  std::memcpy(out->lo, s.lo, sizeof(s.lo));
  std::memcpy(out->hi, s.hi, sizeof(s.hi));
  out->flags = s.flags;
  out->build_ms = s.build_ms;
  return RTMC_OK;
}

rtmc_status rtmc_bvh_download(rtmc_ctx* c, int32_t scene_id, float* nodes, float* tris) {
  rtmc_status st = check_scene(c, scene_id, true);
  if (st) return st;
  const Scene& s = c->scenes[scene_id];
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (nodes && s.n_nodes) HIPCHK(c, hipMemcpy(nodes, s.nodes.p, (size_t)s.n_nodes * 64, hipMemcpyDeviceToHost));
  if (tris && s.n_tris) HIPCHK(c, hipMemcpy(tris, s.tris.p, (size_t)s.n_tris * 48, hipMemcpyDeviceToHost));
  return RTMC_OK;
}

rtmc_status rtmc_bvh_download_wide(rtmc_ctx* c, int32_t scene_id, uint32_t* wide) {
  rtmc_status st = check_scene(c, scene_id, true);
  if (st) return st;
  if (!wide) return fail(c, RTMC_EINVAL, "null pointer");
  const Scene& s = c->scenes[scene_id];
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (s.n_nodes) HIPCHK(c, hipMemcpy(wide, s.nodes4.p, (size_t)s.n_nodes * 64, hipMemcpyDeviceToHost));
  return RTMC_OK;
}

rtmc_status rtmc_load_tables(rtmc_ctx* c, const rtmc_tables* t, int32_t* table_id) {
  if (!c) return RTMC_EINVAL;
  c->err.clear();
  if (!t || !table_id || !t->yield || !t->cdf_E || !t->cdf_F) return fail(c, RTMC_EINVAL, "null pointer");
  if (t->n_E < 2 || t->n_theta < 2 || (int64_t)t->n_E * t->n_theta > kMaxYield)
    return fail(c, RTMC_EINVAL, "yield grid %d x %d out of range", t->n_E, t->n_theta);
  if (t->n_cdf < 2 || t->n_cdf > kMaxCdf) return fail(c, RTMC_EINVAL, "n_cdf %d out of range", t->n_cdf);
  if (!(t->E_min > 0.0) || !(t->E_max > t->E_min) || !std::isfinite(t->E_max) || !std::isfinite(t->Ec) ||
      t->Ec < 0.0)
    return fail(c, RTMC_EINVAL, "bad energy axis or cut-off");
  float ymax = 0.f;
  for (int64_t i = 0; i < (int64_t)t->n_E * t->n_theta; ++i) {
    const float y = t->yield[i];
    if (!finite_f(y) || y < 0.f || y >= 7.f) return fail(c, RTMC_EINVAL, "yield value %lld not in [0, 7)", (long long)i);
    ymax = std::max(ymax, y);
  }
  if (t->emission != RTMC_EMIT_SPECTRUM && t->emission != RTMC_EMIT_PAPER)
    return fail(c, RTMC_EINVAL, "unknown emission mode %d", t->emission);
  if (t->emission == RTMC_EMIT_PAPER) {
    if (!t->esee) return fail(c, RTMC_EINVAL, "the paper's emission rule needs esee");
    for (int64_t i = 0; i < (int64_t)t->n_E * t->n_theta; ++i)
      if (!finite_f(t->esee[i])) return fail(c, RTMC_EINVAL, "esee value %lld not finite", (long long)i);
  }
  if (t->cdf_E[0] != 0.f || t->cdf_F[0] != 0.f || t->cdf_F[t->n_cdf - 1] != 1.f)
    return fail(c, RTMC_EINVAL, "CDF must start at (0, 0) and end at F = 1");
  for (int k = 1; k < t->n_cdf; ++k) {
    if (!finite_f(t->cdf_E[k]) || !(t->cdf_E[k] > t->cdf_E[k - 1]))
      return fail(c, RTMC_EINVAL, "cdf_E must increase strictly (index %d)", k);
    if (!finite_f(t->cdf_F[k]) || t->cdf_F[k] < t->cdf_F[k - 1])
      return fail(c, RTMC_EINVAL, "cdf_F must not decrease (index %d)", k);
  }
  Tables tb;
  tb.nE = t->n_E;
  tb.nth = t->n_theta;
  tb.ncdf = t->n_cdf;
  tb.Emin = t->E_min;
  tb.Emax = t->E_max;
  tb.Ec = t->Ec;
  tb.max_d = std::max(1, (int)std::ceil(ymax));
  tb.emission = t->emission;
  const size_t ny = (size_t)tb.nE * tb.nth;
  const size_t nf = ny + 2 * (size_t)tb.ncdf + (tb.emission == RTMC_EMIT_PAPER ? ny : 0);
  // guide tables of the CDF look-ups (2 x kGuide uint16 = kGuide floats)
  std::vector<float> h(nf + kGuide);
  {
    const int n = tb.ncdf;
    std::vector<uint16_t> gF(kGuide), gE(kGuide);
    // gF[b] = (smallest m >= 1 with cdf_F[m] >= b / kGuide) - 1
    int m = 1;
    for (int b = 0; b < kGuide; ++b) {
      const float tb_ = (float)b / (float)kGuide;
      while (m < n - 1 && !(t->cdf_F[m] >= tb_)) ++m;
      gF[b] = (uint16_t)(m - 1);
    }
    // gE over the bit patterns of positive energies from cdf_E[1] to cdf_E[n - 1]
    uint32_t e1, en;
    std::memcpy(&e1, &t->cdf_E[1], 4);
    std::memcpy(&en, &t->cdf_E[n - 1], 4);
    uint32_t shift = 0;
    while (((en - e1) >> shift) >= (uint32_t)kGuide) ++shift;
    int k = 1;
    for (int b = 0; b < kGuide; ++b) {
      const uint64_t bits = (uint64_t)e1 + ((uint64_t)b << shift);
      float v;
      if (bits >= en) {
        v = t->cdf_E[n - 1];
      } else {
        const uint32_t b32 = (uint32_t)bits;
        std::memcpy(&v, &b32, 4);
      }
      while (k + 1 < n - 1 && t->cdf_E[k + 1] <= v) ++k;
      gE[b] = (uint16_t)k;  // last node at or below v (v >= cdf_E[1])
    }
    tb.e1bits = e1;
    tb.eshift = shift;
    std::memcpy(h.data() + nf, gF.data(), 2 * kGuide);
    std::memcpy(reinterpret_cast<char*>(h.data() + nf) + 2 * kGuide, gE.data(), 2 * kGuide);
  }
  std::memcpy(h.data(), t->yield, sizeof(float) * ny);
  std::memcpy(h.data() + ny, t->cdf_E, sizeof(float) * tb.ncdf);
  std::memcpy(h.data() + ny + tb.ncdf, t->cdf_F, sizeof(float) * tb.ncdf);
  if (tb.emission == RTMC_EMIT_PAPER) std::memcpy(h.data() + ny + 2 * (size_t)tb.ncdf, t->esee, sizeof(float) * ny);
  HIPCHK(c, hipSetDevice(c->device));
  if (ensure(c, tb.buf, h.size() * 4)) return RTMC_ENOMEM;
  HIPCHK(c, hipMemcpyAsync(tb.buf.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->tables.push_back(tb);
  *table_id = (int32_t)c->tables.size() - 1;
  return RTMC_OK;
}

rtmc_status rtmc_trace(rtmc_ctx* c, int32_t scene_id, int32_t table_id, double E_eV, double theta_deg,
                       uint64_t n_primaries, uint64_t seed, const rtmc_trace_opts* opts, rtmc_result* out) {
  rtmc_status st = check_scene(c, scene_id, true);
  if (st) return st;
  c->err.clear();
  if (table_id < 0 || table_id >= (int32_t)c->tables.size()) return fail(c, RTMC_EINVAL, "unknown table id %d", table_id);
  if (!out) return fail(c, RTMC_EINVAL, "null result");
  rtmc_trace_opts o{6, 256, 90, 0, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, 0, nullptr};
  if (opts) {
    o = *opts;
    if (o.n_ebins == 0) o.n_ebins = 256;
    if (o.n_abins == 0) o.n_abins = 90;
  }
  if (o.max_gen < 0 || o.max_gen > kMaxGen) return fail(c, RTMC_EINVAL, "max_gen %d not in [0, 10]", o.max_gen);
  if (o.n_ebins < 1 || o.n_ebins > kMaxEbins || o.n_abins < 1 || o.n_abins > kMaxAbins || o.n_zbins < 0 ||
      o.n_zbins > kMaxZbins)
    return fail(c, RTMC_EINVAL, "histogram bins out of range");
  if (!(E_eV > 0.0) || !std::isfinite(E_eV) || !std::isfinite(theta_deg) || theta_deg > 90.0 || theta_deg < -90.0)
    return fail(c, RTMC_EINVAL, "bad energy or angle");
  if (o.pid0 + n_primaries > 0xFFFFFFFFull) return fail(c, RTMC_EINVAL, "pid0 + n_primaries must stay below 2^32");
  if (o.replay && (o.n_replay < 0 || o.n_replay > 0xFFFFFFFFll || o.replay_gen < 1 || o.replay_gen > o.max_gen))
    return fail(c, RTMC_EINVAL, "replay needs 0 <= n_replay < 2^32 and 1 <= replay_gen <= max_gen");
  if (o.n_replay_out) *o.n_replay_out = 0;
  HIPCHK(c, hipSetDevice(c->device));
  std::vector<HostJob> jobs{{scene_id, E_eV, theta_deg, n_primaries, seed, o.pid0, o.pp_escaped}};
  if (n_primaries == 0) {
    std::memset(out, 0, sizeof(*out));
    if (o.e_hist) std::memset(o.e_hist, 0, 8 * (size_t)o.n_ebins);
    if (o.a_hist) std::memset(o.a_hist, 0, 8 * (size_t)o.n_abins);
    if (o.z_hist && o.n_zbins) std::memset(o.z_hist, 0, 8 * (size_t)o.n_zbins);
    return RTMC_OK;
  }
  TraceOut to;
  c->replay = o.replay && o.n_replay > 0 ? o.replay : nullptr;
  c->n_replay = (uint32_t)o.n_replay;
  c->replay_gen = o.replay_gen;
  st = run_trace(c, table_id, jobs, o.max_gen, o.n_ebins, o.n_abins, o.n_zbins, false, to);
  const bool replayed = c->replay != nullptr;
  c->replay = nullptr;
  if (st) return st;
  if (replayed && o.n_replay_out) {
    uint32_t nr = 0;
    std::memcpy(&nr, static_cast<const char*>(c->pin) + 4, 4);
    *o.n_replay_out = nr;
  }
  fill_result(to.tally.data(), jobs[0], o.n_ebins, o.n_abins, o.n_zbins, o.e_hist, o.a_hist, o.z_hist, to, out);
  return RTMC_OK;
}

rtmc_status rtmc_trace_batch(rtmc_ctx* c, int32_t table_id, const rtmc_job* jobs, int64_t n_jobs, int32_t max_gen,
                             rtmc_result* outs) {
  if (!c) return RTMC_EINVAL;
  c->err.clear();
  if (!jobs || !outs || n_jobs <= 0 || n_jobs > (1 << 27)) return fail(c, RTMC_EINVAL, "bad job list");
  if (table_id < 0 || table_id >= (int32_t)c->tables.size()) return fail(c, RTMC_EINVAL, "unknown table id %d", table_id);
  if (max_gen < 0 || max_gen > kMaxGen) return fail(c, RTMC_EINVAL, "max_gen %d not in [0, 10]", max_gen);
  std::vector<HostJob> hj;
  uint64_t total = 0;
  for (int64_t i = 0; i < n_jobs; ++i) {
    rtmc_status st = check_scene(c, jobs[i].scene_id, true);
    if (st) return st;
    const rtmc_job& j = jobs[i];
    if (!(j.E_eV > 0.0) || !std::isfinite(j.E_eV) || !(std::fabs(j.theta_deg) <= 90.0) ||
        j.n_primaries > 0xFFFFFFFFull)
      return fail(c, RTMC_EINVAL, "job %lld: bad energy, angle or size", (long long)i);
    hj.push_back({j.scene_id, j.E_eV, j.theta_deg, j.n_primaries, j.seed, 0, j.pp_escaped});
    total += j.n_primaries;
  }
  HIPCHK(c, hipSetDevice(c->device));
  if (total == 0) {
    for (int64_t i = 0; i < n_jobs; ++i) std::memset(&outs[i], 0, sizeof(rtmc_result));
    return RTMC_OK;
  }
  // a long sequence of launches (many small chunks) is replayed as a graph;
  // a short one is launched directly, which also times every launch
  const uint64_t n_launch = (uint64_t)plan_chunks(hj, (uint32_t)c->cfg.chunk).size() * (uint64_t)(max_gen + 1);
  TraceOut to;
  rtmc_status st = run_trace(c, table_id, hj, max_gen, 256, 90, 0, n_launch > kGraphLaunches, to);
  if (st) return st;
  const size_t tw = (size_t)T_NCOUNT + 256 + 90;
  for (int64_t i = 0; i < n_jobs; ++i)
    fill_result(to.tally.data() + tw * i, hj[i], 256, 90, 0, nullptr, nullptr, nullptr, to, &outs[i]);
  return RTMC_OK;
}

rtmc_status rtmc_first_hit(rtmc_ctx* c, int32_t scene_id, const float* rays, int64_t n, int32_t* tri_out,
                           float* t_out) {
  rtmc_status st = check_scene(c, scene_id, true);
  if (st) return st;
  c->err.clear();
  if (n < 0 || (n > 0 && (!rays || !tri_out || !t_out))) return fail(c, RTMC_EINVAL, "bad ray arrays");
  if (n >= (int64_t)0xFFFFFFF0) return fail(c, RTMC_EINVAL, "too many rays");
  if (n == 0) return RTMC_OK;
  HIPCHK(c, hipSetDevice(c->device));
  const Scene& s = c->scenes[scene_id];
  const int gdepth = std::max(kGlobalStack, stack_need(s.depth));
  const int block = c->cfg.block;
  const int grid = grid_of(c, c->cfg);
  const size_t waves = (size_t)grid * (block / 64);
  // the 32-bit work counter may run past n by one block claim per wave
  if ((uint64_t)n + (uint64_t)waves * (uint64_t)c->cfg.claim > 0xFFFFFFF0ull) return fail(c, RTMC_EINVAL, "too many rays");
  st = ensure(c, c->gstack, waves * gdepth * 64 * 4);
  if (st) return st;
  // job 0 carries the scene; hit records go to scratch except code and t
  DevJob dj{};
  dj.sc = dev_scene(s);
  DevBuf scratch;
  st = ensure(c, scratch, (size_t)n * 20 + 64 + sizeof(DevJob));
  if (st) return st;
  uint32_t* u = reinterpret_cast<uint32_t*>(scratch.p);
  DevJob* djd = reinterpret_cast<DevJob*>(u + 5 * (size_t)n + 16);
  hipError_t e = hipMemcpyAsync(djd, &dj, sizeof(dj), hipMemcpyHostToDevice, c->stream);
  TraverseArgs ta{};
  ta.jobs = djd;
  ta.n_jobs = 1;
  ta.src = 2;
  ta.rays = rays;
  ta.count = (uint32_t)n;
  ta.hit.code = tri_out;
  ta.hit.t = t_out;
  ta.hit.f0 = reinterpret_cast<float*>(u);
  ta.hit.f1 = reinterpret_cast<float*>(u + n);
  ta.hit.visits = u + 2 * (size_t)n;
  ta.hit.tests = u + 3 * (size_t)n;
  ta.hit.wraps = u + 4 * (size_t)n;
  ta.work = u + 5 * (size_t)n;
  ta.err = ta.work + 1;
  ta.gstack = reinterpret_cast<uint32_t*>(c->gstack.p);
  ta.lds_stack = c->cfg.lds_stack;
  ta.gstack_depth = gdepth;
  ta.refill = c->cfg.refill;
  ta.claim_max = (uint32_t)c->cfg.claim;
  if (e == hipSuccess) e = launch_fill_u32(ta.work, 0u, 2, c->stream);
  if (e == hipSuccess) e = launch_traverse(ta, false, c->cfg.occupancy, grid, block, c->stream);
  if (e == hipSuccess)
    e = launch_hit_ids(reinterpret_cast<const float4*>(s.tris.p), tri_out, n, tri_out, c->stream);
  // the scratch is released only after the launches that use it have finished
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(c, scratch);
  if (e != hipSuccess) return fail(c, RTMC_EDEVICE, "first hit: %s", hipGetErrorString(e));
  return RTMC_OK;
}

rtmc_status rtmc_first_hit_noalloc(rtmc_ctx* c, int32_t scene_id, const float* rays, int64_t n, int32_t* tri_out,
                                   float* t_out) {
  rtmc_status st = check_scene(c, scene_id, true);
  if (st) return st;
  c->err.clear();
  if (n < 0 || (n > 0 && (!rays || !tri_out || !t_out))) return fail(c, RTMC_EINVAL, "bad ray arrays");
  if (n > kNoAllocMaxRays)
    return fail(c, RTMC_EINVAL, "%lld rays exceed the %lld one call without allocation takes", (long long)n,
                (long long)kNoAllocMaxRays);
  if (!c->scratch) return fail(c, RTMC_ESTATE, "no scratch memory on device %d", c->device);
  if (n == 0) return RTMC_OK;
  HIPCHK(c, hipSetDevice(c->device));
  const Scene& s = c->scenes[scene_id];
  const rtmc_launch_cfg& cfg = c->cfg;
  if (traverse_lds_bytes(cfg.lds_stack, cfg.block) > c->lds_per_block)
    return fail(c, RTMC_EINVAL, "launch shape needs more LDS than a workgroup has");
  // global stack entries beyond the LDS part: exactly what the tree can need
  const int gdepth = std::max(8, stack_need(s.depth) - cfg.lds_stack);
  const int wpb = cfg.block / 64;
  const size_t wave_bytes = (size_t)gdepth * 64 * 4;
  // as many persistent workgroups as the launch shape asks for and the stack region holds
  const int grid = (int)std::min<size_t>((size_t)grid_of(c, cfg), kScratchStack / (wave_bytes * wpb));
  if (grid < 1) return fail(c, RTMC_EINVAL, "BVH of depth %d too deep for the scratch stack", s.depth);
  unsigned char* base = static_cast<unsigned char*>(c->scratch);
  uint32_t* head = reinterpret_cast<uint32_t*>(base);
  DevJob* djd = reinterpret_cast<DevJob*>(base + 256);
  uint32_t* u = reinterpret_cast<uint32_t*>(base + kScratchHead);
  const size_t M = (size_t)kNoAllocMaxRays;
  DevJob dj{};
  dj.sc = dev_scene(s);
  TraverseArgs ta{};
  ta.jobs = djd;
  ta.n_jobs = 1;
  ta.src = 2;
  ta.rays = rays;
  ta.count = (uint32_t)n;
  ta.hit.code = tri_out;
  ta.hit.t = t_out;
  ta.hit.f0 = reinterpret_cast<float*>(u);
  ta.hit.f1 = reinterpret_cast<float*>(u + M);
  ta.hit.visits = u + 2 * M;
  ta.hit.tests = u + 3 * M;
  ta.hit.wraps = u + 4 * M;
  ta.work = head;
  ta.err = head + 1;
  ta.gstack = u + 5 * M;
  ta.lds_stack = cfg.lds_stack;
  ta.gstack_depth = gdepth;
  ta.refill = cfg.refill;
  ta.claim_max = (uint32_t)cfg.claim;
  HIPCHK(c, launch_store_job(djd, dj, c->stream));
  HIPCHK(c, launch_fill_u32(head, 0u, 2, c->stream));
  HIPCHK(c, launch_traverse(ta, false, cfg.occupancy, grid, cfg.block, c->stream));
  HIPCHK(c, launch_hit_ids(reinterpret_cast<const float4*>(s.tris.p), tri_out, n, tri_out, c->stream));
  return RTMC_OK;
}

rtmc_status rtmc_sort_pairs_u64(rtmc_ctx* c, uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits) {
  if (!c) return RTMC_EINVAL;
  c->err.clear();
  if (n < 0 || (n > 0 && (!keys || !vals)) || key_bits < 1 || key_bits > 64 || n >= (int64_t)0xFFFFFFFF)
    return fail(c, RTMC_EINVAL, "bad sort arguments");
  if (n <= 1) return RTMC_OK;
  HIPCHK(c, hipSetDevice(c->device));
  DevBuf k2, v2, h;
  if (ensure(c, k2, (size_t)n * 8) || ensure(c, v2, (size_t)n * 4) || ensure(c, h, radix_hist_words(n) * 4)) {
    dev_free(c, k2);
    dev_free(c, v2);
    dev_free(c, h);
    return RTMC_ENOMEM;
  }
  bool alt = false;
  hipError_t e = radix_sort_pairs(keys, vals, reinterpret_cast<uint64_t*>(k2.p), reinterpret_cast<uint32_t*>(v2.p),
                                  reinterpret_cast<uint32_t*>(h.p), n, key_bits, c->stream, &alt);
  if (e == hipSuccess && alt) {
    e = hipMemcpyAsync(keys, k2.p, (size_t)n * 8, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(vals, v2.p, (size_t)n * 4, hipMemcpyDeviceToDevice, c->stream);
  }
  // scratch is released only after the work that uses it has finished
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(c, k2);
  dev_free(c, v2);
  dev_free(c, h);
  if (e != hipSuccess) return fail(c, RTMC_EDEVICE, "sort: %s", hipGetErrorString(e));
  return RTMC_OK;
}

rtmc_status rtmc_set_launch(rtmc_ctx* c, const rtmc_launch_cfg* cfg) {
  if (!c) return RTMC_EINVAL;
  if (!cfg || cfg->block < 64 || cfg->block > 256 || cfg->block % 64 || cfg->wg_per_cu < 1 || cfg->wg_per_cu > 64 ||
      cfg->lds_stack < 4 || cfg->lds_stack > 64 || cfg->chunk < 1 || cfg->refill < 1 || cfg->refill > 64 ||
      cfg->claim < 0 || cfg->claim > kClaimLimit || (cfg->claim > 0 && cfg->claim < 64))
    return fail(c, RTMC_EINVAL, "bad launch shape");
  c->cfg = *cfg;
  if (c->cfg.claim == 0) c->cfg.claim = kClaimDefault;
  return RTMC_OK;
}

rtmc_status rtmc_get_launch(rtmc_ctx* c, rtmc_launch_cfg* cfg) {
  if (!c || !cfg) return RTMC_EINVAL;
  *cfg = c->cfg;
  return RTMC_OK;
}

constexpr double kTuneMargin = 0.02;  // relative gain a launch-shape change must show on the probe

rtmc_status rtmc_autotune(rtmc_ctx* c, int32_t scene_id, int32_t table_id, double E_eV, double theta_deg,
                          uint64_t n_primaries, rtmc_launch_cfg* best) {
  rtmc_status st = check_scene(c, scene_id, true);
  if (st) return st;
  if (table_id < 0 || table_id >= (int32_t)c->tables.size()) return fail(c, RTMC_EINVAL, "unknown table id %d", table_id);
  if (n_primaries == 0 || n_primaries > 0xFFFFFFFFull) return fail(c, RTMC_EINVAL, "bad calibration size");
  const TuneKey key = tune_key(c, scene_id, table_id, E_eV, theta_deg, n_primaries);
  {
    std::lock_guard<std::mutex> lock(tune_mu);
    for (const auto& e : tune_cache)
      if (e.first == key) {
        c->cfg = e.second;
        if (best) *best = e.second;
        return RTMC_OK;
      }
  }
  const rtmc_launch_cfg keep = c->cfg;
  // coordinate search: one knob at a time, starting from the current shape
  rtmc_launch_cfg cur = keep;
  auto time_cfg = [&](const rtmc_launch_cfg& cf, double* ms) -> rtmc_status {
    if (traverse_lds_bytes(cf.lds_stack, cf.block) > c->lds_per_block) {
      *ms = 1e30;
      return RTMC_OK;
    }
    c->cfg = cf;
    rtmc_result r;
    rtmc_status s2 = rtmc_trace(c, scene_id, table_id, E_eV, theta_deg, n_primaries, 12345, nullptr, &r);
    *ms = s2 ? 1e30 : r.ms;
    return s2;
  };
  double best_ms = 1e30;
  st = time_cfg(cur, &best_ms);
  if (st) {
    c->cfg = keep;
    return st;
  }
  // chunk candidates: halves, quarters, eighths of the calibration trace.  Any
  // chunk of at least its length traces it as one chunk, so the probe cannot
  // tell such chunks apart: the current one (usually far larger, as a batch
  // needs) is the baseline and is never replaced by an equivalent of the
  // probe's own length.
  std::vector<int32_t> chunks;
  for (int k = 1; k < 4; ++k) {
    const uint64_t ch = n_primaries >> k;
    if (ch >= 4096) chunks.push_back((int32_t)std::min<uint64_t>(ch, 1u << 30));
  }
  const std::vector<std::vector<int32_t>> knobs = {
      {64, 128, 256},                    // block
      {2, 4, 6, 7, 8, 12, 16},           // workgroups per CU (of 256 threads)
      {8, 12, 16, 24, 32},               // LDS stack entries
      {24, 32, 40, 48, 56, 64},          // refill threshold
      {0, 6, 8},                         // kernel build
      {512, 1024, 2048, 4096, 8192},     // rays per wave per claim
      chunks};                           // primaries per chunk
  for (int pass = 0; pass < 2; ++pass) {
    for (size_t knob = 0; knob < knobs.size(); ++knob) {
      for (const int32_t v : knobs[knob]) {
        rtmc_launch_cfg cf = cur;
        if (knob == 0) {
          cf.block = v;
          cf.wg_per_cu = std::max(1, cur.wg_per_cu * cur.block / v);
        }
        if (knob == 1) cf.wg_per_cu = v * 256 / cf.block;
        if (knob == 2) cf.lds_stack = v;
        if (knob == 3) cf.refill = v;
        if (knob == 4) cf.occupancy = v;
        if (knob == 5) cf.claim = v;
        if (knob == 6) cf.chunk = v;
        if (cf.wg_per_cu < 1 || cf.wg_per_cu > 64) continue;
        if (std::memcmp(&cf, &cur, sizeof(cf)) == 0) continue;
        double ms;
        st = time_cfg(cf, &ms);
        if (st) {
          c->cfg = keep;
          return st;
        }
        // a change must win by more than the probe's timing noise
        if (ms < best_ms * (1.0 - kTuneMargin)) {
          best_ms = ms;
          cur = cf;
        }
      }
    }
  }
  c->cfg = cur;
  {
    std::lock_guard<std::mutex> lock(tune_mu);
    tune_cache.emplace_back(key, cur);
  }
  if (best) *best = cur;
  return RTMC_OK;
}

rtmc_status rtmc_copy_probe(rtmc_ctx* c, void* dst, const void* src, size_t bytes, int32_t reps, double* ms) {
  if (!c) return RTMC_EINVAL;
  if (!dst || !src || bytes < 16 || bytes % 16 || reps < 1 || !ms) return fail(c, RTMC_EINVAL, "bad probe arguments");
  HIPCHK(c, hipSetDevice(c->device));
  const int grid = c->n_cu * 16;
  HIPCHK(c, launch_copy_probe(reinterpret_cast<float4*>(dst), reinterpret_cast<const float4*>(src), bytes / 16, grid,
                              c->stream));
  HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  for (int r = 0; r < reps; ++r)
    HIPCHK(c, launch_copy_probe(reinterpret_cast<float4*>(dst), reinterpret_cast<const float4*>(src), bytes / 16,
                                grid, c->stream));
  HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float t = 0.f;
  HIPCHK(c, hipEventElapsedTime(&t, c->ev0, c->ev1));
  *ms = t / reps;
  return RTMC_OK;
}


}  // extern "C"

// ---------------------------------------------------------------- surrogate
namespace {

constexpr int kPadIn = 32;  // first-layer inputs padded to one MFMA k-step

// offsets (floats) into the padded FP32 parameter vector
struct SrgLayout {
  int64_t W[5], b[5], wout, bout, total;
};

SrgLayout srg_layout(const Surrogate& g) {
  SrgLayout L{};
  int64_t o = 0;
  for (int l = 1; l <= g.depth; ++l) {
    const int kin = l == 1 ? kPadIn : g.width;
    L.W[l] = o;
    o += (int64_t)g.width * kin;
    L.b[l] = o;
    o += g.width;
  }
  L.wout = o;
  o += g.width;
  L.bout = o;
  o += 1;
  L.total = o;
  return L;
}

// BF16 weight copies: per layer W_l [width x kin] then W_l^T [kin x width]
int64_t srg_wbf_off(const Surrogate& g, int l, bool transposed) {
  int64_t o = 0;
  for (int q = 1; q < l; ++q) o += 2 * (int64_t)g.width * (q == 1 ? kPadIn : g.width);
  const int kin = l == 1 ? kPadIn : g.width;
  return o + (transposed ? (int64_t)g.width * kin : 0);
}

rtmc_status srg_check(rtmc_ctx* c, int32_t id) {
  if (!c) return RTMC_EINVAL;
  c->err.clear();
  if (id < 0 || id >= (int32_t)c->srgs.size()) return fail(c, RTMC_EINVAL, "unknown surrogate id %d", id);
  return RTMC_OK;
}

rtmc_status srg_refresh_bf16(rtmc_ctx* c, Surrogate& g) {
  const SrgLayout L = srg_layout(g);
  const float* m = reinterpret_cast<const float*>(g.master.p);
  __bf16* wb = reinterpret_cast<__bf16*>(g.wbf.p);
  for (int l = 1; l <= g.depth; ++l) {
    const int kin = l == 1 ? kPadIn : g.width;
    HIPCHK(c, mlp_to_bf16(m + L.W[l], g.width, kin, wb + srg_wbf_off(g, l, false), wb + srg_wbf_off(g, l, true),
                          c->stream));
  }
  return RTMC_OK;
}

// ---- fused training (mlp.hip): per pass of at most kTrainChunk rows one
// mlp_train_rows and one mlp_train_dw, then one mlp_train_update
struct SrgTrainWs {
  float *part, *loss_part, *zbuf, *acc;
  __bf16 *gt, *ht;
  int grid, ldk;
};

rtmc_status srg_train_ws(rtmc_ctx* c, Surrogate& g, int64_t batch, SrgTrainWs& w) {
  if (mlp_train_lds_bytes() > c->lds_per_block)
    return fail(c, RTMC_ENOTIMPL, "surrogate training needs %zu bytes of LDS per workgroup (device limit %zu)",
                mlp_train_lds_bytes(), c->lds_per_block);
  const int ldk = (int)std::min<int64_t>(batch, kTrainChunk);
  const int grid = mlp_train_grid(ldk);  // the first pass is the largest
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t o_loss = up((size_t)grid * kTrainSmall * 4), o_z = o_loss + up((size_t)kTrainMaxWg * 4);
  const size_t o_gt = o_z + up((size_t)grid * 3 * kTrainRows * 256 * 4);
  const size_t o_ht = o_gt + up((size_t)4 * 256 * ldk * 2), o_acc = o_ht + up((size_t)(32 + 3 * 256) * ldk * 2);
  const size_t total = o_acc + 256;
  rtmc_status st = ensure(c, g.tws, total);
  if (st) return st;
  char* b = static_cast<char*>(g.tws.p);
  w.part = reinterpret_cast<float*>(b);
  w.loss_part = reinterpret_cast<float*>(b + o_loss);
  w.zbuf = reinterpret_cast<float*>(b + o_z);
  w.gt = reinterpret_cast<__bf16*>(b + o_gt);
  w.ht = reinterpret_cast<__bf16*>(b + o_ht);
  w.acc = reinterpret_cast<float*>(b + o_acc);
  w.grid = grid;
  w.ldk = ldk;
  return RTMC_OK;
}

MlpTrain srg_train_args(const Surrogate& g, const SrgTrainWs& w, int64_t batch) {
  const SrgLayout L = srg_layout(g);
  const __bf16* wb = reinterpret_cast<const __bf16*>(g.wbf.p);
  MlpTrain t{};
  t.master = reinterpret_cast<const float*>(g.master.p);
  for (int l = 1; l <= 4; ++l) {
    t.W[l - 1] = wb + srg_wbf_off(g, l, false);
    t.Wt[l - 1] = wb + srg_wbf_off(g, l, true);
    t.off_b[l - 1] = L.b[l];
  }
  t.off_wout = L.wout;
  t.off_bout = L.bout;
  t.batch = (int)batch;
  t.n_in = g.n_in;
  t.zbuf = w.zbuf;
  t.gt = w.gt;
  t.ht = w.ht;
  t.ldk = w.ldk;
  t.part = w.part;
  t.loss_part = w.loss_part;
  return t;
}

// The gradient of the batch into g.grad and its loss into w.acc[0]: the
// passes of mlp_train_rows and mlp_train_dw in row order.
rtmc_status srg_gradient_passes(rtmc_ctx* c, Surrogate& g, const SrgTrainWs& w, MlpTrain t,
                                const MlpDw* loop = nullptr) {
  const SrgLayout L = srg_layout(g);
  MlpDw d{};
  if (loop) d = *loop;  // the device loop's step bookkeeping
  d.gt = w.gt;
  d.ht = w.ht;
  d.ldk = w.ldk;
  d.grad = reinterpret_cast<float*>(g.grad.p);
  for (int l = 1; l <= 4; ++l) {
    d.off_W[l - 1] = L.W[l];
    d.off_b[l - 1] = L.b[l];
  }
  d.off_wout = L.wout;
  d.off_bout = L.bout;
  d.part = w.part;
  d.loss_part = w.loss_part;
  d.n_part = w.grid;
  d.acc = w.acc;
  for (int64_t r0 = 0; r0 < t.batch; r0 += w.ldk) {
    t.row0 = (int)r0;
    t.rows = (int)std::min<int64_t>(w.ldk, t.batch - r0);
    t.first_pass = r0 == 0;
    HIPCHK(c, mlp_train_rows(t, c->stream));
    d.rows = t.rows;
    d.first_pass = t.first_pass;
    d.last_pass = r0 + t.rows >= t.batch;
    HIPCHK(c, mlp_train_dw(d, c->stream));
  }
  return RTMC_OK;
}

// AdamW on the masters from g.grad and the BF16 copies of W and W^T.
MlpUpdate srg_update_args(Surrogate& g) {
  const SrgLayout L = srg_layout(g);
  __bf16* wb = reinterpret_cast<__bf16*>(g.wbf.p);
  MlpUpdate u{};
  u.n_par = L.total;
  u.grad = reinterpret_cast<const float*>(g.grad.p);
  u.p = reinterpret_cast<float*>(g.master.p);
  u.m = reinterpret_cast<float*>(g.mom1.p);
  u.v = reinterpret_cast<float*>(g.mom2.p);
  u.b1 = 0.9f;
  u.b2 = 0.999f;
  u.eps = 1e-8f;
  for (int l = 1; l <= 4; ++l) {
    u.Wb[l - 1] = wb + srg_wbf_off(g, l, false);
    u.Wtb[l - 1] = wb + srg_wbf_off(g, l, true);
    u.off_W[l - 1] = L.W[l];
    u.kin[l - 1] = l == 1 ? kPadIn : g.width;
  }
  return u;
}

void pub_to_pad(const Surrogate& g, const float* pub, std::vector<float>& pad) {
  const SrgLayout L = srg_layout(g);
  pad.assign((size_t)L.total, 0.0f);
  int64_t o = 0;
  for (int l = 1; l <= g.depth; ++l) {
    const int kin = l == 1 ? g.n_in : g.width;
    const int kp = l == 1 ? kPadIn : g.width;
    for (int r = 0; r < g.width; ++r)
      for (int k = 0; k < kin; ++k) pad[(size_t)(L.W[l] + (int64_t)r * kp + k)] = pub[o++];
    for (int r = 0; r < g.width; ++r) pad[(size_t)(L.b[l] + r)] = pub[o++];
  }
  for (int r = 0; r < g.width; ++r) pad[(size_t)(L.wout + r)] = pub[o++];
  pad[(size_t)L.bout] = pub[o++];
}

void pad_to_pub(const Surrogate& g, const float* pad, float* pub) {
  const SrgLayout L = srg_layout(g);
  int64_t o = 0;
  for (int l = 1; l <= g.depth; ++l) {
    const int kin = l == 1 ? g.n_in : g.width;
    const int kp = l == 1 ? kPadIn : g.width;
    for (int r = 0; r < g.width; ++r)
      for (int k = 0; k < kin; ++k) pub[o++] = pad[(size_t)(L.W[l] + (int64_t)r * kp + k)];
    for (int r = 0; r < g.width; ++r) pub[o++] = pad[(size_t)(L.b[l] + r)];
  }
  for (int r = 0; r < g.width; ++r) pub[o++] = pad[(size_t)(L.wout + r)];
  pub[o++] = pad[(size_t)L.bout];
}

rtmc_status srg_upload(rtmc_ctx* c, Surrogate& g, const std::vector<float>& pad) {
  HIPCHK(c, hipMemcpyAsync(g.master.p, pad.data(), pad.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_fill_u32(reinterpret_cast<uint32_t*>(g.mom1.p), 0u, pad.size(), c->stream));
  HIPCHK(c, launch_fill_u32(reinterpret_cast<uint32_t*>(g.mom2.p), 0u, pad.size(), c->stream));
  g.step = 0;
  rtmc_status st = srg_refresh_bf16(c, g);
  if (st) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RTMC_OK;
}

}  // namespace

extern "C" {

rtmc_status rtmc_srg_create(rtmc_ctx* c, int32_t n_in, int32_t width, int32_t depth, uint64_t seed, int32_t* id) {
  if (!c) return RTMC_EINVAL;
  c->err.clear();
  if (!id || n_in < 1 || n_in > kPadIn) return fail(c, RTMC_EINVAL, "n_in must be in [1, 32]");
  if (width != 256 || depth != 4) return fail(c, RTMC_ENOTIMPL, "only width 256 and depth 4 are built");
  HIPCHK(c, hipSetDevice(c->device));
  Surrogate g;
  g.n_in = n_in;
  g.width = width;
  g.depth = depth;
  const SrgLayout L = srg_layout(g);
  g.n_pad = L.total;
  g.n_pub = L.total - (int64_t)width * (kPadIn - n_in);
  if (ensure(c, g.master, L.total * 4) || ensure(c, g.mom1, L.total * 4) || ensure(c, g.mom2, L.total * 4) ||
      ensure(c, g.grad, L.total * 4) || ensure(c, g.wbf, (size_t)srg_wbf_off(g, depth + 1, false) * 2)) {
    dev_free(c, g.master);
    dev_free(c, g.mom1);
    dev_free(c, g.mom2);
    dev_free(c, g.grad);
    dev_free(c, g.wbf);
    return RTMC_ENOMEM;
  }
  // He-uniform initialisation from a seeded 64-bit generator (host)
  std::vector<float> pub((size_t)g.n_pub, 0.0f);
  uint64_t st = seed ^ 0x9E3779B97F4A7C15ull;
  auto next = [&]() {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  int64_t o = 0;
  for (int l = 1; l <= depth; ++l) {
    const int kin = l == 1 ? n_in : width;
    const double a = std::sqrt(6.0 / kin);
    for (int64_t i = 0; i < (int64_t)width * kin; ++i) pub[(size_t)o++] = (float)((2.0 * next() - 1.0) * a);
    o += width;  // zero bias
  }
  const double a = std::sqrt(3.0 / width);
  for (int r = 0; r < width; ++r) pub[(size_t)o++] = (float)((2.0 * next() - 1.0) * a);
  c->srgs.push_back(g);
  Surrogate& gg = c->srgs.back();
  std::vector<float> pad;
  pub_to_pad(gg, pub.data(), pad);
  rtmc_status s2 = srg_upload(c, gg, pad);
  if (s2) return s2;
  *id = (int32_t)c->srgs.size() - 1;
  return RTMC_OK;
}

rtmc_status rtmc_srg_param_count(rtmc_ctx* c, int32_t id, int64_t* n) {
  rtmc_status st = srg_check(c, id);
  if (st) return st;
  if (!n) return fail(c, RTMC_EINVAL, "null output");
  *n = c->srgs[id].n_pub;
  return RTMC_OK;
}

rtmc_status rtmc_srg_get_params(rtmc_ctx* c, int32_t id, float* params, int64_t n) {
  rtmc_status st = srg_check(c, id);
  if (st) return st;
  Surrogate& g = c->srgs[id];
  if (!params || n != g.n_pub) return fail(c, RTMC_EINVAL, "parameter array must hold %lld floats", (long long)g.n_pub);
  HIPCHK(c, hipSetDevice(c->device));
  std::vector<float> pad((size_t)g.n_pad);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(pad.data(), g.master.p, pad.size() * 4, hipMemcpyDeviceToHost));
  pad_to_pub(g, pad.data(), params);
  return RTMC_OK;
}

rtmc_status rtmc_srg_set_params(rtmc_ctx* c, int32_t id, const float* params, int64_t n) {
  rtmc_status st = srg_check(c, id);
  if (st) return st;
  Surrogate& g = c->srgs[id];
  if (!params || n != g.n_pub) return fail(c, RTMC_EINVAL, "parameter array must hold %lld floats", (long long)g.n_pub);
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return fail(c, RTMC_EINVAL, "parameter %lld is not finite", (long long)i);
  HIPCHK(c, hipSetDevice(c->device));
  std::vector<float> pad;
  pub_to_pad(g, params, pad);
  return srg_upload(c, g, pad);
}

rtmc_status rtmc_srg_gradient(rtmc_ctx* c, int32_t id, const float* X, const float* y, int64_t batch, float* loss,
                              float* grads) {
  rtmc_status st = srg_check(c, id);
  if (st) return st;
  Surrogate& g = c->srgs[id];
  if (!X || !y || batch < 32 || batch % 32 || batch > (1 << 22)) return fail(c, RTMC_EINVAL, "batch must be a positive multiple of 32");
  HIPCHK(c, hipSetDevice(c->device));
  SrgTrainWs w;
  st = srg_train_ws(c, g, batch, w);
  if (st) return st;
  MlpTrain t = srg_train_args(g, w, batch);
  t.x = X;
  t.t = y;
  st = srg_gradient_passes(c, g, w, t);
  if (st) return st;
  float acc = 0.f;
  HIPCHK(c, hipMemcpyAsync(&acc, w.acc, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (loss) *loss = acc;
  if (grads) {
    std::vector<float> pad((size_t)g.n_pad);
    HIPCHK(c, hipMemcpy(pad.data(), g.grad.p, pad.size() * 4, hipMemcpyDeviceToHost));
    pad_to_pub(g, pad.data(), grads);
  }
  return RTMC_OK;
}

rtmc_status rtmc_srg_train_step(rtmc_ctx* c, int32_t id, const float* X, const float* y, int64_t batch, float lr,
                                float weight_decay, float* loss) {
  rtmc_status st = srg_check(c, id);
  if (st) return st;
  Surrogate& g = c->srgs[id];
  if (!X || !y || batch < 32 || batch % 32 || batch > (1 << 22)) return fail(c, RTMC_EINVAL, "batch must be a positive multiple of 32");
  if (!(lr > 0.0f) || !(weight_decay >= 0.0f)) return fail(c, RTMC_EINVAL, "bad learning rate or weight decay");
  HIPCHK(c, hipSetDevice(c->device));
  SrgTrainWs w;
  st = srg_train_ws(c, g, batch, w);
  if (st) return st;
  MlpTrain t = srg_train_args(g, w, batch);
  t.x = X;
  t.t = y;
  st = srg_gradient_passes(c, g, w, t);
  if (st) return st;
  g.step += 1;
  MlpUpdate u = srg_update_args(g);
  u.lr = lr;
  u.wd = weight_decay;
  u.c1 = 1.0f - (float)std::pow((double)u.b1, (double)g.step);
  u.c2 = 1.0f - (float)std::pow((double)u.b2, (double)g.step);
  HIPCHK(c, mlp_train_update(u, c->stream));
  if (loss) {
    float acc = 0.f;
    HIPCHK(c, hipMemcpyAsync(&acc, w.acc, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *loss = acc;
  }
  return RTMC_OK;
}

rtmc_status rtmc_srg_train(rtmc_ctx* c, int32_t id, const float* X, const float* y, int64_t n, int64_t batch,
                           int32_t steps, const float* lr, float weight_decay, uint64_t seed, int32_t use_graph,
                           float* losses) {
  rtmc_status st = srg_check(c, id);
  if (st) return st;
  Surrogate& g = c->srgs[id];
  if (!X || !y || !lr || n < 1 || n > 0xFFFFFFFFll) return fail(c, RTMC_EINVAL, "bad training arrays");
  if (batch < 32 || batch % 32 || batch > (1 << 22)) return fail(c, RTMC_EINVAL, "batch must be a positive multiple of 32");
  if (steps < 1 || steps > (1 << 24)) return fail(c, RTMC_EINVAL, "steps must be in [1, 2^24]");
  if (!(weight_decay >= 0.0f)) return fail(c, RTMC_EINVAL, "bad weight decay");
  for (int32_t s = 0; s < steps; ++s)
    if (!(lr[s] > 0.0f) || !std::isfinite(lr[s])) return fail(c, RTMC_EINVAL, "learning rate %d not positive", s);
  HIPCHK(c, hipSetDevice(c->device));
  SrgTrainWs w;
  st = srg_train_ws(c, g, batch, w);
  if (st) return st;
  // loop buffer: 2 state words and the step's 3 AdamW constants (padded to
  // 256 B), lr[steps], losses[steps]
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t o_lr = 256, o_loss = o_lr + up((size_t)steps * 4), total = o_loss + up((size_t)steps * 4);
  st = ensure(c, g.tbuf, total);
  if (st) return st;
  char* base = static_cast<char*>(g.tbuf.p);
  uint32_t* state = reinterpret_cast<uint32_t*>(base);
  float* sched = reinterpret_cast<float*>(base + 64);
  float* lr_d = reinterpret_cast<float*>(base + o_lr);
  float* loss_d = reinterpret_cast<float*>(base + o_loss);
  HIPCHK(c, hipMemcpyAsync(lr_d, lr, (size_t)steps * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_fill_u32(state, (uint32_t)g.step, 2, c->stream));
  MlpTrain targs = srg_train_args(g, w, batch);
  targs.src_x = X;
  targs.src_t = y;
  targs.n_src = (uint32_t)n;
  targs.seed = seed;
  targs.state = state;
  MlpUpdate uargs = srg_update_args(g);
  uargs.sched = sched;
  uargs.wd = weight_decay;
  MlpDw loop{};
  loop.state = state;
  loop.losses = loss_d;
  loop.lr_sched = lr_d;
  loop.sched = sched;
  loop.b1 = uargs.b1;
  loop.b2 = uargs.b2;
  // one step: rows drawn on the device, forward, backward signals and the
  // weight gradients (per pass of rows; the last pass also records the loss
  // and advances the step), AdamW and the BF16 weights
  auto one_step = [&]() -> rtmc_status {
    rtmc_status s2 = srg_gradient_passes(c, g, w, targs, &loop);
    if (s2) return s2;
    HIPCHK(c, mlp_train_update(uargs, c->stream));
    return RTMC_OK;
  };
  if (!use_graph) {
    for (int32_t s = 0; s < steps; ++s) {
      st = one_step();
      if (st) return st;
    }
  } else {
    uint32_t wd_bits;
    std::memcpy(&wd_bits, &weight_decay, 4);
    const std::vector<uint64_t> key = {(uint64_t)(uintptr_t)X, (uint64_t)(uintptr_t)y, (uint64_t)n, (uint64_t)batch,
                                       seed, (uint64_t)(uintptr_t)g.tbuf.p, (uint64_t)(uintptr_t)g.tws.p,
                                       (uint64_t)(uintptr_t)g.master.p, (uint64_t)steps, wd_bits};
    // the step runs on the context's own capture stream, ordered after the work above
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->gstream, c->ev0, 0));
    if (!g.tgexec || key != g.tkey) {
      if (g.tgexec) {
        (void)hipGraphExecDestroy(g.tgexec);
        g.tgexec = nullptr;
      }
      hipStream_t saved = c->stream;
      c->stream = c->gstream;
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) {
        c->stream = saved;
        return fail(c, RTMC_EDEVICE, "graph capture: %s", hipGetErrorString(e));
      }
      st = one_step();
      e = hipStreamEndCapture(c->gstream, &graph);
      c->stream = saved;
      if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      HIPCHK(c, e);
      e = hipGraphInstantiate(&g.tgexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIPCHK(c, e);
      g.tkey = key;
    }
    for (int32_t s = 0; s < steps; ++s) HIPCHK(c, hipGraphLaunch(g.tgexec, c->gstream));
    HIPCHK(c, hipEventRecord(c->ev1, c->gstream));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev1, 0));
  }
  g.step += steps;
  if (losses) HIPCHK(c, hipMemcpyAsync(losses, loss_d, (size_t)steps * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RTMC_OK;
}

rtmc_status rtmc_srg_predict(rtmc_ctx* c, int32_t id, const float* X, int64_t n, float* y) {
  rtmc_status st = srg_check(c, id);
  if (st) return st;
  Surrogate& g = c->srgs[id];
  if (n < 0 || (n > 0 && (!X || !y))) return fail(c, RTMC_EINVAL, "bad prediction arrays");
  if (n == 0) return RTMC_OK;
  HIPCHK(c, hipSetDevice(c->device));
  // one fused kernel: activations stay in LDS, no workspace
  const SrgLayout L = srg_layout(g);
  const float* m = reinterpret_cast<const float*>(g.master.p);
  const __bf16* wb = reinterpret_cast<const __bf16*>(g.wbf.p);
  MlpInfer q{};
  q.x = X;
  q.n = n;
  q.n_in = g.n_in;
  for (int l = 1; l <= 4; ++l) {
    q.W[l - 1] = wb + srg_wbf_off(g, l, false);
    q.bias[l - 1] = m + L.b[l];
  }
  q.wout = m + L.wout;
  q.bout = m + L.bout;
  q.y = y;
  HIPCHK(c, mlp_infer(q, c->stream));
  return RTMC_OK;
}

}  // extern "C"

