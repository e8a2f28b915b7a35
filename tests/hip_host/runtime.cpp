// Runtime of the host build: one fiber per lane (started with ucontext, switched with
// setjmp/longjmp), wavefront exchanges between the blocked lanes of a wave, the blocks of a
// launch spread over a pool of host threads (each runs whole blocks, with its own fibers and
// its own copy of the workgroup-shared arrays), and device allocations that end at a guard page
// and are unmapped for good when freed, so any access past the end of a buffer or after its
// release faults at once; the fault handler names the allocation the address belongs to.
#include "hip/hip_runtime.h"

#include <atomic>
#include <condition_variable>
#include <csetjmp>
#include <csignal>
#include <dlfcn.h>
#include <execinfo.h>
#include <map>
#include <mutex>
#include <thread>
#include <sys/mman.h>
#include <ucontext.h>
#include <unistd.h>

struct EmuStream { bool capturing = false; std::vector<std::function<void()>> rec; };
struct EmuGraph { std::vector<std::function<void()>> ops; };
struct EmuGraphExec { std::vector<std::function<void()>> ops; };

namespace emu {
namespace {
constexpr size_t kStack = 256 << 10;
struct Lane {
  jmp_buf ctx;
  ucontext_t uc;
  char* stack = nullptr;
  dim3 tid;
  int t = 0;
  bool done = false, blocked = false;
  int kind = 0;
  uint64_t val = 0, res = 0;
  int a = 0, b = 0, c = 0, d = 0;
  void* ra = nullptr;  // call site of the pending wavefront operation
  void* bt[10] = {};   // its call chain, kept when TACCEL_HOST_TRACE is set
  int nbt = 0;
};
const bool g_trace = getenv("TACCEL_HOST_TRACE") != nullptr;
thread_local std::vector<Lane> g_lanes;
thread_local Lane* g_cur = nullptr;
thread_local jmp_buf g_sched;
thread_local ucontext_t g_tmp;
thread_local dim3 g_bidx;
dim3 g_bdim, g_gdim;
thread_local const std::function<void()>* g_body = nullptr;
const dim3 g_host_tid(0, 0, 0);

void trampoline() {
  Lane* L = g_cur;
  if (_setjmp(L->ctx) == 0) _longjmp(g_sched, 1);
  (*g_body)();
  g_cur->done = true;
  _longjmp(g_sched, 1);
}

void resume(Lane* L) {
  g_cur = L;
  if (_setjmp(g_sched) == 0) _longjmp(L->ctx, 1);
}

[[noreturn]] void die(const char* m) {
  fprintf(stderr, "host build FATAL: %s\n", m);
  fflush(stderr);
  abort();
}

// A wavefront operation that the wave's lanes do not meet together: name every lane's state
// and the function it waits in, then stop.
[[noreturn]] void die_wave(const char* m, const Lane* any) {
  fprintf(stderr, "host build FATAL: %s (block %u,%u,%u)\n", m, g_bidx.x, g_bidx.y, g_bidx.z);
  const int w0 = any->t & ~63;
  for (int i = w0; i < std::min<int>((int)g_lanes.size(), w0 + 64); ++i) {
    const Lane& L = g_lanes[i];
    Dl_info info{};
    const bool found = L.ra && dladdr(L.ra, &info);
    const char* fn = found && info.dli_sname ? info.dli_sname : "?";
    const long off = found ? (long)((char*)L.ra - (char*)info.dli_fbase) : 0;
    fprintf(stderr, "  lane %d: done=%d kind=%d a=%d in %s (+0x%lx)", i & 63, (int)L.done, L.kind, L.a, fn, off);
    for (int k = 1; k < L.nbt; ++k)
      if (dladdr(L.bt[k], &info)) fprintf(stderr, " <- +0x%lx", (long)((char*)L.bt[k] - (char*)info.dli_fbase));
    fprintf(stderr, "\n");
  }
  fflush(stderr);
  abort();
}

void resolve_group(std::vector<Lane*>& grp) {
  const int kind = grp[0]->kind;
  Lane* by_lane[64] = {nullptr};
  for (Lane* L : grp) by_lane[L->t & 63] = L;
  if (kind == OP_WAVEBAR) return;
  if (kind == OP_BALLOT || kind == OP_ALL) {
    uint64_t m = 0;
    bool all = true;
    for (Lane* L : grp) {
      if (L->val) m |= 1ull << (L->t & 63);
      all = all && L->val;
    }
    for (Lane* L : grp) L->res = kind == OP_BALLOT ? m : (all ? 1 : 0);
    return;
  }
  for (Lane* L : grp) {
    const int lane = L->t & 63;
    if (kind == OP_SHFL || kind == OP_SHFL_XOR || kind == OP_SHFL_UP) {
      const int w = L->b, seg = lane & ~(w - 1);
      int src;
      if (kind == OP_SHFL) src = seg + (L->a & (w - 1));
      else if (kind == OP_SHFL_XOR) src = lane ^ L->a;
      else src = lane - L->a;
      // a source outside the segment reads the lane's own value; an inactive source lane
      // holds no defined value on the hardware, so reading one is a bug
      if (src < seg || src >= seg + w) L->res = L->val;
      else if (!by_lane[src]) die_wave("shuffle reads an inactive lane", L);
      else L->res = by_lane[src]->val;
    } else if (kind == OP_READFIRST) {
      int first = 0;
      while (!by_lane[first]) ++first;
      L->res = by_lane[first]->val & 0xffffffffull;
    } else if (kind == OP_READLANE) {
      if (!by_lane[L->a]) die_wave("readlane of an inactive lane", L);
      L->res = by_lane[L->a]->val & 0xffffffffull;
    } else if (kind == OP_DPP) {
      const uint32_t old = (uint32_t)(L->val >> 32);
      const int ctrl = L->a, row_mask = L->b, bank_mask = L->c;
      const bool bound = L->d != 0;
      const int row = lane >> 4, i = lane & 15;
      if (!((row_mask >> row) & 1) || !((bank_mask >> (i >> 2)) & 1)) {
        L->res = old;
        continue;
      }
      int src = -1;
      if (ctrl >= 0x111 && ctrl <= 0x11f) {
        const int n = ctrl - 0x110;
        if (i - n >= 0) src = lane - n;
      } else if (ctrl == 0x142) {
        if (row >= 1) src = row * 16 - 1;
      } else if (ctrl == 0x143) {
        if (row >= 2) src = 31;
      } else {
        die("unsupported DPP control");
      }
      if (src < 0) {
        L->res = bound ? 0 : old;
      } else if (!by_lane[src]) {
        die_wave("DPP reads an inactive lane", L);
      } else {
        L->res = by_lane[src]->val & 0xffffffffull;
      }
    }
  }
}

void run_block(const std::function<void()>& body) {
  const int n = (int)(g_bdim.x * g_bdim.y * g_bdim.z);
  if ((int)g_lanes.size() < n) g_lanes.resize(n);
  g_body = &body;
  for (int i = 0; i < n; ++i) {
    Lane& L = g_lanes[i];
    if (!L.stack) {
      L.stack = (char*)mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
      if (L.stack == MAP_FAILED) die("stack mmap");
    }
    L.t = i;
    L.tid = dim3(i % g_bdim.x, (i / g_bdim.x) % g_bdim.y, i / (g_bdim.x * g_bdim.y));
    L.done = L.blocked = false;
    getcontext(&L.uc);
    L.uc.uc_stack.ss_sp = L.stack;
    L.uc.uc_stack.ss_size = kStack;
    L.uc.uc_link = nullptr;
    makecontext(&L.uc, trampoline, 0);
    g_cur = &L;
    if (_setjmp(g_sched) == 0) swapcontext(&g_tmp, &L.uc);
  }
  for (;;) {
    for (int i = 0; i < n; ++i) {
      Lane& L = g_lanes[i];
      if (!L.done && !L.blocked) resume(&L);
    }
    bool live = false, progressed = false;
    const int nw = (n + 63) / 64;
    for (int w = 0; w < nw; ++w) {
      // fast path: every waiting lane of the wave at the same kind of op with the same params
      {
        Lane* first = nullptr;
        bool same = true, any_sync = false;
        static thread_local std::vector<Lane*> grp;
        grp.clear();
        for (int i = 64 * w; i < std::min(n, 64 * w + 64); ++i) {
          Lane& L = g_lanes[i];
          if (L.done) continue;
          live = true;
          if (L.kind == OP_SYNC) { any_sync = true; continue; }
          if (!first) first = &L;
          else if (L.kind != first->kind || L.a != first->a || L.b != first->b || L.c != first->c || L.d != first->d) same = false;
          grp.push_back(&L);
        }
        if (!first) continue;
        if (same && (first->kind != OP_SHFL || true)) {
          (void)any_sync;
          resolve_group(grp);
          for (Lane* L : grp) L->blocked = false;
          progressed = true;
          continue;
        }
      }
      std::map<std::vector<int>, std::vector<Lane*>> groups;
      for (int i = 64 * w; i < std::min(n, 64 * w + 64); ++i) {
        Lane& L = g_lanes[i];
        if (L.done) continue;
        live = true;
        if (L.kind == OP_SYNC) continue;
        std::vector<int> key = {L.kind};
        if (L.kind == OP_SHFL || L.kind == OP_SHFL_XOR || L.kind == OP_SHFL_UP) key.push_back(L.b);
        if (L.kind == OP_DPP) { key.push_back(L.a); key.push_back(L.b); key.push_back(L.c); key.push_back(L.d); }
        if (L.kind == OP_READLANE) key.push_back(L.a);
        groups[key].push_back(&L);
      }
      for (auto& kv : groups) {
        resolve_group(kv.second);
        for (Lane* L : kv.second) L->blocked = false;
        progressed = true;
      }
    }
    if (!live) break;
    if (progressed) continue;
    // every live lane waits at the workgroup barrier
    for (int i = 0; i < n; ++i)
      if (!g_lanes[i].done) g_lanes[i].blocked = false;
  }
  g_cur = nullptr;
}
}  // namespace

const dim3& tidx() { return g_cur ? g_cur->tid : g_host_tid; }
const dim3& bidx() { return g_bidx; }
const dim3& bdim() { return g_bdim; }
const dim3& gdim() { return g_gdim; }

uint64_t lane_op(int kind, uint64_t val, int a, int b, int c, int d, int e) {
  (void)e;
  Lane* L = g_cur;
  if (!L) die("lane op outside a kernel");
  L->kind = kind;
  L->val = val;
  L->a = a; L->b = b; L->c = c; L->d = d;
  L->ra = __builtin_return_address(0);
  if (g_trace) L->nbt = backtrace(L->bt, 10);
  L->blocked = true;
  if (_setjmp(L->ctx) == 0) _longjmp(g_sched, 1);
  return L->res;
}

// Blocks of one launch are taken in turn by the calling thread and the pool's workers.
struct Pool {
  std::mutex m;
  std::condition_variable cv, done_cv;
  std::vector<std::thread> workers;
  uint64_t gen = 0;
  int busy = 0;
  std::atomic<long long> next{0};
  long long nblocks = 0;
  const std::function<void()>* body = nullptr;
  dim3 grid;

  static int size() {
    const char* e = getenv("TACCEL_HOST_THREADS");
    int n = e ? atoi(e) : (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(n, 64));
  }
  void work() {
    for (long long i; (i = next.fetch_add(1)) < nblocks;) {
      g_bidx = dim3((unsigned)(i % grid.x), (unsigned)((i / grid.x) % grid.y),
                    (unsigned)(i / ((long long)grid.x * grid.y)));
      run_block(*body);
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] { return gen != seen; });
        seen = gen;
      }
      work();
      std::lock_guard<std::mutex> lk(m);
      if (--busy == 0) done_cv.notify_all();
    }
  }
  void run(dim3 g, const std::function<void()>& b) {
    const long long n = (long long)g.x * g.y * g.z;
    if (workers.empty()) {
      const int k = size() - 1;
      for (int i = 0; i < k; ++i) {
        workers.emplace_back([this] { loop(); });
        workers.back().detach();
      }
    }
    if (n <= 1 || workers.empty()) {
      for (long long i = 0; i < n; ++i) {
        g_bidx = dim3((unsigned)(i % g.x), (unsigned)((i / g.x) % g.y), (unsigned)(i / ((long long)g.x * g.y)));
        run_block(b);
      }
      return;
    }
    {
      std::lock_guard<std::mutex> lk(m);
      grid = g;
      body = &b;
      nblocks = n;
      next = 0;
      busy = (int)workers.size();
      ++gen;
    }
    cv.notify_all();
    work();
    std::unique_lock<std::mutex> lk(m);
    done_cv.wait(lk, [&] { return busy == 0; });
  }
};
Pool& g_pool = *new Pool;  // never destroyed: its detached workers wait on it until exit

static void run_grid(dim3 grid, dim3 block, const std::function<void()>& body) {
  g_gdim = grid;
  g_bdim = block;
  g_pool.run(grid, body);
}

// Kernels of host threads that share the runtime (the server's cohorts) run one at a time.
std::recursive_mutex g_exec;

void launch(hipStream_t s, dim3 grid, dim3 block, std::function<void()> body) {
  if (s && s->capturing) {
    s->rec.push_back([grid, block, body]() { run_grid(grid, block, body); });
    return;
  }
  std::lock_guard<std::recursive_mutex> lk(g_exec);
  run_grid(grid, block, body);
}
}  // namespace emu

// ---------------------------------------------------------------- memory
namespace {
struct Region { char* base; size_t total; bool freed; };
std::map<void*, Region> g_regions;
struct Tag { size_t n; int serial; };
std::map<void*, Tag> g_tags;
int g_serial = 0;

const size_t kPage = 4096;

std::mutex g_alloc;

void* guarded(size_t n) {
  std::lock_guard<std::mutex> lk(g_alloc);
  const size_t n16 = (std::max<size_t>(n, 1) + 15) & ~size_t(15);
  const size_t data = (n16 + kPage - 1) & ~(kPage - 1);
  const size_t total = kPage + data + kPage;
  char* base = (char*)mmap(nullptr, total, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
  if (base == MAP_FAILED) return nullptr;
  mprotect(base, kPage, PROT_NONE);
  mprotect(base + kPage + data, kPage, PROT_NONE);
  char* p = base + kPage + data - n16;
  std::memset(p, 0x7F, n16);
  g_regions[p] = {base, total, false};
  g_tags[p] = {n, ++g_serial};
  return p;
}
hipError_t release(void* p) {
  if (!p) return hipSuccess;
  std::lock_guard<std::mutex> lk(g_alloc);
  auto it = g_regions.find(p);
  if (it == g_regions.end()) { fprintf(stderr, "host build: free of unknown pointer %p\n", p); abort(); }
  if (it->second.freed) { fprintf(stderr, "host build: double free %p\n", p); abort(); }
  it->second.freed = true;
  mprotect(it->second.base, it->second.total, PROT_NONE);
  return hipSuccess;
}
}  // namespace

namespace {
void on_segv(int, siginfo_t* si, void*) {
  char* a = (char*)si->si_addr;
  fprintf(stderr, "host build: memory fault at %p\n", (void*)a);
  for (auto& kv : g_regions) {
    const Region& r = kv.second;
    if (a >= r.base && a < r.base + r.total) {
      const Tag& t = g_tags[kv.first];
      fprintf(stderr, "  in region of allocation #%d ptr %p size %zu freed=%d offset from ptr %td\n", t.serial,
              kv.first, t.n, (int)r.freed, a - (char*)kv.first);
    }
  }
  void* bt[64];
  const int nb = backtrace(bt, 64);
  backtrace_symbols_fd(bt, nb, 2);
  _exit(139);
}
struct Installer {
  Installer() {
    static char altstack[1 << 16];
    stack_t ss{};
    ss.ss_sp = altstack;
    ss.ss_size = sizeof(altstack);
    sigaltstack(&ss, nullptr);
    struct sigaction sa{};
    sa.sa_sigaction = on_segv;
    sa.sa_flags = SA_SIGINFO | SA_ONSTACK;
    sigaction(SIGSEGV, &sa, nullptr);
  }
} g_installer;
}  // namespace

hipError_t hipMalloc(void** p, size_t n) { *p = guarded(n); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipFree(void* p) { return release(p); }
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = guarded(n); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipHostFree(void* p) { return release(p); }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { if (n) std::memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { if (n) std::memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { if (n) std::memset(d, v, n); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new EmuStream(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new EmuEvent(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new EmuEvent(); return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "emulated error"; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) { s->capturing = true; s->rec.clear(); return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  *g = new EmuGraph{s->rec};
  s->rec.clear();
  s->capturing = false;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) { *e = new EmuGraphExec{g->ops}; return hipSuccess; }
hipError_t hipGraphExecUpdate(hipGraphExec_t e, hipGraph_t g, hipGraphNode_t*, hipGraphExecUpdateResult* r) { e->ops = g->ops; *r = hipGraphExecUpdateSuccess; return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  std::lock_guard<std::recursive_mutex> lk(emu::g_exec);
  for (auto& f : e->ops) f();
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }
