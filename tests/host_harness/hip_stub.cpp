// Host-only stand-in for the HIP runtime, used to exercise the library's host
// orchestration (stream forks and joins, graph capture and the graph cache,
// solver chunk loops, the batched step) on the CPU under AddressSanitizer.
//
// Device memory is host memory (calloc), so every copy the library makes is
// bounds-checked by the sanitizer.  Kernels are not run: a launch only checks
// its configuration and is recorded on its stream.  The stand-in models the
// stream-ordering and capture rules of the HIP/CUDA graph API and counts every
// breach as a violation:
//   * destroying an executable graph that is still in flight, or launching a
//     destroyed one;
//   * a captured stream waiting on an event recorded outside the capture, a
//     stream waiting on an event whose last record was inside a capture that
//     has ended, or two captures joined through an event;
//   * a capture that ends while a stream forked into it has work not joined
//     back, or synchronising / allocating calls while a capture is active;
//   * a memset recorded into a capture (a fill kernel is required instead);
//   * a launch with an empty or oversized grid, block or LDS request.
// Device-to-host copies of at most 64 bytes into pinned memory are taken as
// reads of the solver's open-system counters and receive scripted values (a
// seeded sequence of counts, all zero with probability 0.3), so that the host
// loops see many different sets of open jobs.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <vector>

struct ihipGraph;
struct hipGraphExec;
struct ihipStream_t;
struct ihipEvent_t;

namespace {

struct Item {
  unsigned long long seq = 0;
  hipGraphExec *exec = nullptr;      // a graph launch
  ihipStream_t *dep = nullptr;       // or a wait on dep's work up to dep_seq
  unsigned long long dep_seq = 0;
};

// State is built on first use: the library's module constructors register
// their device variables before this file's globals would be constructed.
struct State {
  std::recursive_mutex mu;
  long long violations = 0, launches = 0, graph_launches = 0, instantiated = 0, exec_destroyed = 0;
  long long count_reads = 0, captures = 0;
  std::mt19937_64 rng{12345};
  std::set<void *> pinned;
  std::map<void *, size_t> dev;               // fake device allocations and their sizes
  std::map<const void *, void *> symbols;     // __device__ variables -> fake storage
  std::map<const void *, size_t> symbol_size;
  int active_captures = 0;
};
State &st() {
  static State *s = new State();
  return *s;
}
#define g_mu (st().mu)
#define g_violations (st().violations)
#define g_launches (st().launches)
#define g_graph_launches (st().graph_launches)
#define g_instantiated (st().instantiated)
#define g_exec_destroyed (st().exec_destroyed)
#define g_count_reads (st().count_reads)
#define g_captures (st().captures)
#define g_rng (st().rng)
#define g_pinned (st().pinned)
#define g_dev (st().dev)
#define g_symbols (st().symbols)
#define g_symbol_size (st().symbol_size)
#define g_active_captures (st().active_captures)

void violation(const char *what) {
  ++g_violations;
  std::fprintf(stderr, "[hip-stub] VIOLATION: %s\n", what);
}

}  // namespace

struct ihipGraph {
  bool ended = false, destroyed = false;
  long long nodes = 0;
  ihipStream_t *origin = nullptr;
  std::set<ihipStream_t *> joined;
};

struct hipGraphExec {
  bool destroyed = false;
  int inflight = 0;
  long long nodes = 0;
};

struct ihipStream_t {
  unsigned long long seq = 0;
  std::vector<Item> pending;
  ihipGraph *capturing = nullptr;
  unsigned long long ops_in_capture = 0;   // operations recorded while captured
  unsigned long long joined_back_at = ~0ull;
};

struct ihipEvent_t {
  bool recorded = false;
  ihipGraph *capture = nullptr;   // graph the last record was captured into
  ihipStream_t *src = nullptr;
  unsigned long long seq = 0;
  unsigned long long src_ops = 0; // ops_in_capture of src at a captured record
};

namespace {

ihipStream_t &null_stream() {
  static ihipStream_t *s = new ihipStream_t();
  return *s;
}
std::set<ihipStream_t *> &streams() {
  static std::set<ihipStream_t *> *s = new std::set<ihipStream_t *>{&null_stream()};
  return *s;
}
#define g_null_stream (null_stream())
#define g_streams (streams())

ihipStream_t *S(hipStream_t s) { return s ? s : &g_null_stream; }

void complete(ihipStream_t *s, unsigned long long upto) {
  std::vector<Item> keep, done;
  for (const Item &it : s->pending) (it.seq <= upto ? done : keep).push_back(it);
  s->pending.swap(keep);
  for (const Item &it : done) {
    if (it.exec) --it.exec->inflight;
    if (it.dep) complete(it.dep, it.dep_seq);
  }
}

void complete_all() {
  for (ihipStream_t *s : g_streams) complete(s, ~0ull);
}

// One operation enqueued on s: a captured node, or an ordered item.
unsigned long long enqueue(ihipStream_t *s) {
  if (s->capturing) {
    ++s->capturing->nodes;
    ++s->ops_in_capture;
  }
  return ++s->seq;
}

void no_capture_active(const char *call) {
  if (g_active_captures > 0) {
    std::string m = std::string(call) + " called while a stream capture is active";
    violation(m.c_str());
  }
}

}  // namespace

extern "C" {

// ---- registration of kernels and device variables (no device code here)
void **__hipRegisterFatBinary(const void *) {
  static void *module = nullptr;
  return &module;
}
void __hipUnregisterFatBinary(void **) {}
void __hipRegisterFunction(void **, const void *, char *, const char *, unsigned int, uint3 *, uint3 *, dim3 *, dim3 *,
                           int *) {}
void __hipRegisterVar(void **, void *var, char *, char *, int, size_t size, int, int) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_symbol_size[var] = size;
}

hipError_t __hipPushCallConfiguration(dim3, dim3, size_t, hipStream_t);
hipError_t __hipPopCallConfiguration(dim3 *, dim3 *, size_t *, hipStream_t *);
}

namespace {
struct CallCfg {
  dim3 grid, block;
  size_t shmem;
  hipStream_t stream;
};
thread_local std::vector<CallCfg> t_cfg;

void check_launch(dim3 grid, dim3 block, size_t shmem) {
  const unsigned long long thr = (unsigned long long)block.x * block.y * block.z;
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) violation("kernel launch with an empty grid");
  if (grid.y > 65535 || grid.z > 65535 || grid.x > 2147483647u) violation("kernel launch with an oversized grid");
  if (thr == 0 || thr > 1024) violation("kernel launch with an empty or oversized block");
  if (shmem > 160 * 1024) violation("kernel launch asking for more than 160 KB of LDS");
}
}  // namespace

extern "C" {

hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shmem, hipStream_t stream) {
  t_cfg.push_back({grid, block, shmem, stream});
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3 *grid, dim3 *block, size_t *shmem, hipStream_t *stream) {
  if (t_cfg.empty()) return hipErrorInvalidValue;
  const CallCfg c = t_cfg.back();
  t_cfg.pop_back();
  *grid = c.grid;
  *block = c.block;
  *shmem = c.shmem;
  *stream = c.stream;
  return hipSuccess;
}

hipError_t hipLaunchKernel(const void *, dim3 grid, dim3 block, void **, size_t shmem, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  check_launch(grid, block, shmem);
  ++g_launches;
  enqueue(S(stream));
  return hipSuccess;
}

const char *hipGetErrorName(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "hipErrorStub"; }
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}

// ---- memory
hipError_t hipMalloc(void **p, size_t n) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture_active("hipMalloc");
  *p = std::calloc(1, n ? n : 1);
  if (!*p) return hipErrorOutOfMemory;
  g_dev[*p] = n;
  return hipSuccess;
}
hipError_t hipFree(void *p) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture_active("hipFree");
  if (!p) return hipSuccess;
  complete_all();   // hipFree synchronises the device
  if (!g_dev.erase(p)) violation("hipFree of a pointer that is not a device allocation");
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture_active("hipHostMalloc");
  *p = std::calloc(1, n ? n : 1);
  if (!*p) return hipErrorOutOfMemory;
  g_pinned.insert(*p);
  return hipSuccess;
}
hipError_t hipHostFree(void *p) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!p) return hipSuccess;
  complete_all();
  if (!g_pinned.erase(p)) violation("hipHostFree of a pointer that is not pinned memory");
  std::free(p);
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **dev, const void *symbol) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  auto it = g_symbols.find(symbol);
  if (it == g_symbols.end()) {
    auto sz = g_symbol_size.find(symbol);
    if (sz == g_symbol_size.end()) return hipErrorInvalidSymbol;
    void *p = std::calloc(1, sz->second);
    g_dev[p] = sz->second;
    it = g_symbols.emplace(symbol, p).first;
  }
  *dev = it->second;
  return hipSuccess;
}

static void do_copy(void *dst, const void *src, size_t n, hipMemcpyKind kind) {
  const bool counts = kind == hipMemcpyDeviceToHost && g_pinned.count(dst) && n <= 64 && n % 4 == 0;
  if (counts) {
    // scripted open-system counts of the solver's chunk loop
    ++g_count_reads;
    int *c = (int *)dst;
    const bool none = std::uniform_real_distribution<double>(0, 1)(g_rng) < 0.3;
    for (size_t i = 0; i < n / 4; ++i) c[i] = none ? 0 : (int)(g_rng() % 3);
    return;
  }
  std::memmove(dst, src, n);
}

hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind kind) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture_active("hipMemcpy");
  complete(&g_null_stream, ~0ull);
  do_copy(dst, src, n, kind);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind kind, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  ihipStream_t *s = S(stream);
  if (s->capturing && (kind == hipMemcpyDeviceToHost || kind == hipMemcpyHostToDevice))
    violation("host copy recorded into a stream capture");
  enqueue(s);
  do_copy(dst, src, n, kind);
  return hipSuccess;
}
hipError_t hipMemset(void *dst, int v, size_t n) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture_active("hipMemset");
  std::memset(dst, v, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  ihipStream_t *s = S(stream);
  if (s->capturing) violation("memset recorded into a stream capture");
  enqueue(s);
  std::memset(dst, v, n);
  return hipSuccess;
}

// ---- streams and events
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  *s = new ihipStream_t();
  g_streams.insert(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!s || !g_streams.count(s)) {
    violation("hipStreamDestroy of an unknown stream");
    return hipErrorInvalidValue;
  }
  if (s->capturing) violation("hipStreamDestroy of a stream inside a capture");
  complete(s, ~0ull);
  g_streams.erase(s);
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  ihipStream_t *s = S(stream);
  if (s->capturing) violation("hipStreamSynchronize on a capturing stream");
  no_capture_active("hipStreamSynchronize");
  complete(s, s->seq);
  return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture_active("hipDeviceSynchronize");
  complete_all();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int) {
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  ihipStream_t *s = S(stream);
  e->recorded = true;
  e->src = s;
  if (s->capturing) {
    e->capture = s->capturing;
    ++s->capturing->nodes;
    ++s->ops_in_capture;
    e->src_ops = s->ops_in_capture;
  } else {
    e->capture = nullptr;
    e->seq = s->seq;
  }
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t stream, hipEvent_t e, unsigned int) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  ihipStream_t *t = S(stream);
  if (!e->recorded) return hipSuccess;
  if (e->capture) {
    ihipGraph *g = e->capture;
    if (g->ended) {
      violation("wait on an event whose last record was inside a capture that has ended");
      return hipErrorInvalidValue;
    }
    if (!t->capturing) {       // fork: t joins the capture
      t->capturing = g;
      t->ops_in_capture = 0;
      t->joined_back_at = ~0ull;
      g->joined.insert(t);
    } else if (t->capturing != g) {
      violation("two stream captures joined through an event");
      return hipErrorInvalidValue;
    }
    // join back: the recording stream has done nothing since the record
    if (e->src != t && e->src->capturing == g && e->src->ops_in_capture == e->src_ops)
      e->src->joined_back_at = e->src_ops;
    ++g->nodes;
    ++t->ops_in_capture;
    return hipSuccess;
  }
  if (t->capturing) {
    violation("a captured stream waits on an event recorded outside the capture");
    return hipErrorInvalidValue;
  }
  Item it;
  it.seq = ++t->seq;
  it.dep = e->src;
  it.dep_seq = e->seq;
  t->pending.push_back(it);
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture_active("hipEventSynchronize");
  if (e->capture) violation("hipEventSynchronize on an event recorded inside a capture");
  if (e->recorded && !e->capture) complete(e->src, e->seq);
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
  *ms = 1.0f;
  return hipSuccess;
}

// ---- graphs
hipError_t hipStreamBeginCapture(hipStream_t stream, hipStreamCaptureMode) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  ihipStream_t *s = S(stream);
  if (s->capturing) {
    violation("hipStreamBeginCapture on a stream already capturing");
    return hipErrorInvalidValue;
  }
  ihipGraph *g = new ihipGraph();
  g->origin = s;
  s->capturing = g;
  s->ops_in_capture = 0;
  ++g_active_captures;
  ++g_captures;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t stream, hipGraph_t *graph) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  ihipStream_t *s = S(stream);
  ihipGraph *g = s->capturing;
  if (!g || g->origin != s) {
    violation("hipStreamEndCapture on a stream that did not begin a capture");
    return hipErrorInvalidValue;
  }
  for (ihipStream_t *t : g->joined) {
    if (t->joined_back_at != t->ops_in_capture) violation("capture ended with a forked stream not joined back");
    t->capturing = nullptr;
  }
  s->capturing = nullptr;
  g->ended = true;
  --g_active_captures;
  *graph = g;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t graph, hipGraphNode_t *, char *, size_t) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!graph || !graph->ended || graph->destroyed) {
    violation("hipGraphInstantiate of a graph that is not a finished capture");
    return hipErrorInvalidValue;
  }
  hipGraphExec *x = new hipGraphExec();
  x->nodes = graph->nodes;
  *exec = x;
  ++g_instantiated;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t graph) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!graph || graph->destroyed) violation("hipGraphDestroy of a destroyed graph");
  else graph->destroyed = true;   // kept (ended) so that stale capture events can still be recognised
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!exec || exec->destroyed) {
    violation("hipGraphLaunch of a destroyed executable graph");
    return hipErrorInvalidValue;
  }
  ihipStream_t *s = S(stream);
  if (s->capturing) violation("graph launched into a stream capture");
  Item it;
  it.seq = enqueue(s);
  it.exec = exec;
  ++exec->inflight;
  s->pending.push_back(it);
  ++g_graph_launches;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!exec || exec->destroyed) {
    violation("hipGraphExecDestroy of a destroyed executable graph");
    return hipErrorInvalidValue;
  }
  if (exec->inflight > 0) violation("hipGraphExecDestroy of an executable graph still in flight");
  exec->destroyed = true;   // kept, so that a later launch of it is detected
  ++g_exec_destroyed;
  return hipSuccess;
}

// ---- report for the driver
void hip_stub_report(long long *out) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  out[0] = g_violations;
  out[1] = g_launches;
  out[2] = g_graph_launches;
  out[3] = g_instantiated;
  out[4] = g_exec_destroyed;
  out[5] = g_count_reads;
  out[6] = g_captures;
}

}  // extern "C"
