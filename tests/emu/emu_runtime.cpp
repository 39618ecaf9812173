// The CPU emulation of the HIP runtime declared in include/hip/hip_runtime.h (test
// infrastructure only): synchronous memory, stream and event calls, and kernel launches
// that run every workgroup as a set of host threads.
#include <hip/hip_runtime.h>

#include <sanitizer/asan_interface.h>

#include <barrier>
#include <deque>
#include <map>
#include <algorithm>
#include <condition_variable>
#include <semaphore>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

thread_local EmuIdx threadIdx, blockIdx, blockDim, gridDim;

namespace fm {
// the dynamic LDS of the kernels (extern __shared__ char smem[] in namespace fm)
constexpr size_t kEmuLds = 160 * 1024;
alignas(256) char smem[kEmuLds];
}  // namespace fm

struct EmuEvent {
  unsigned flags;
  bool done = true;   // recorded work has run
  long pending = 0;   // markers of this event still queued
};
struct EmuStream {
  unsigned flags;
  // an operation, or a wait for an event (op empty, wait set)
  struct Op {
    std::function<void()> op;
    EmuEvent* wait = nullptr;
  };
  std::deque<Op> q;
};

namespace {
std::recursive_mutex g_launch;
EmuStream g_null{0, {}};
std::vector<EmuStream*> g_streams{&g_null};  // in creation order
std::map<const char*, size_t> g_pinned;  // pinned allocations: start, bytes
EmuStream* str(hipStream_t s) { return s ? s : &g_null; }

// Run queued work until `until` holds: repeatedly the front operation of the most
// recently created stream whose front is runnable (a wait is runnable once its event is
// done).  Returns false if nothing can run while the condition still fails.
template <class C>
bool drain(C until) {
  std::lock_guard<std::recursive_mutex> lock(g_launch);
  while (!until()) {
    bool ran = false;
    for (auto it = g_streams.rbegin(); it != g_streams.rend() && !ran; ++it) {
      EmuStream* st = *it;
      if (st->q.empty()) continue;
      EmuStream::Op op = std::move(st->q.front());
      if (op.wait && !op.wait->done) {
        st->q.front() = std::move(op);
        continue;
      }
      st->q.pop_front();
      if (op.op) op.op();
      ran = true;
    }
    if (!ran) return false;
  }
  return true;
}
bool all_idle() {
  for (EmuStream* s : g_streams)
    if (!s->q.empty()) return false;
  return true;
}
void drain_all() {
  if (!drain(all_idle)) std::fprintf(stderr, "emu: queued work waits on an event never recorded\n");
}
void enqueue(hipStream_t s, std::function<void()> f) {
  std::lock_guard<std::recursive_mutex> lock(g_launch);
  str(s)->q.push_back({std::move(f), nullptr});
}
// The wavefront barrier.  Lanes of a wavefront run in lockstep on the device, so lanes
// that branch around a wave barrier (an early return from a wave-synchronous helper)
// simply do not take part in it.  Here a lane waiting at the workgroup barrier, or
// finished, is "parked" and counts as arrived at every wave barrier of its wavefront
// until the workgroup barrier releases it; the workgroup barrier's completion step
// (which runs before any thread is released) unparks the live lanes.
struct WaveBar {
  std::mutex m;
  std::condition_variable cv;
  int size, arrived = 0, parked = 0, exited = 0;
  long gen = 0;
  explicit WaveBar(int n) : size(n) {}
  void complete_if_ready() {
    if (arrived > 0 && arrived + parked >= size) {
      arrived = 0;
      ++gen;
      cv.notify_all();
    }
  }
  void wait() {
    std::unique_lock<std::mutex> lock(m);
    const long g = gen;
    ++arrived;
    complete_if_ready();
    cv.wait(lock, [&] { return gen != g; });
  }
  void park() {
    std::lock_guard<std::mutex> lock(m);
    ++parked;
    complete_if_ready();
  }
  void exit() {
    std::lock_guard<std::mutex> lock(m);
    ++parked;
    ++exited;
    complete_if_ready();
  }
  void unpark_all() {  // the workgroup barrier completed
    std::lock_guard<std::mutex> lock(m);
    parked = exited;
  }
};
struct UnparkWaves {
  std::vector<std::unique_ptr<WaveBar>>* waves;
  void operator()() noexcept {
    for (auto& w : *waves) w->unpark_all();
  }
};
using BlockBar = std::barrier<UnparkWaves>;
thread_local BlockBar* t_block = nullptr;
thread_local WaveBar* t_wave = nullptr;
hipError_t g_last = hipSuccess;
constexpr int kEmuCUs = 4;
}  // namespace

namespace emu {
namespace {
// Workers that play the threads of a workgroup, reused across workgroups and launches:
// worker t waits on its own semaphore, runs the body of the current block as thread t,
// leaves the block's barriers and counts itself done.
struct Pool {
  struct Block {
    const std::function<void()>* body;
    dim3 grid, block, idx;
    BlockBar* wg;
    std::vector<std::unique_ptr<WaveBar>>* waves;
  };
  std::vector<std::unique_ptr<std::binary_semaphore>> go;
  std::vector<std::thread> workers;
  Block cur{};
  std::mutex mu;
  std::condition_variable cv;
  int remaining = 0;
  bool stop = false;

  // room for the largest workgroup up front: workers index go[] while it grows
  Pool() {
    go.reserve(1024);
    workers.reserve(1024);
  }
  void grow(int n) {
    while ((int)workers.size() < n) {
      const int t = (int)workers.size();
      go.emplace_back(new std::binary_semaphore(0));
      workers.emplace_back([this, t]() { work(t); });
    }
  }
  void work(int t) {
    for (;;) {
      go[t]->acquire();
      if (stop) return;
      const Block b = cur;
      threadIdx = {(unsigned)(t % b.block.x), (unsigned)((t / b.block.x) % b.block.y),
                   (unsigned)(t / (b.block.x * b.block.y))};
      blockIdx = {b.idx.x, b.idx.y, b.idx.z};
      blockDim = {b.block.x, b.block.y, b.block.z};
      gridDim = {b.grid.x, b.grid.y, b.grid.z};
      t_block = b.wg;
      t_wave = (*b.waves)[t / 64].get();
      (*b.body)();
      t_wave->exit();
      t_block->arrive_and_drop();
      std::lock_guard<std::mutex> lock(mu);
      if (--remaining == 0) cv.notify_one();
    }
  }
  void run(const Block& b, int n) {
    grow(n);
    cur = b;
    {
      std::lock_guard<std::mutex> lock(mu);
      remaining = n;
    }
    for (int t = 0; t < n; ++t) go[t]->release();
    std::unique_lock<std::mutex> lock(mu);
    cv.wait(lock, [this] { return remaining == 0; });
  }
  ~Pool() {
    stop = true;
    for (auto& g : go) g->release();
    for (auto& w : workers) w.join();
  }
};
Pool g_pool;
}  // namespace

void run_grid(dim3 grid, dim3 block, size_t lds_bytes, const std::function<void()>& body);

void launch(hipStream_t s, dim3 grid, dim3 block, size_t lds_bytes, std::function<void()> body) {
  const int n = (int)(block.x * block.y * block.z);
  if (n < 1 || n > 1024 || lds_bytes > fm::kEmuLds || grid.x < 1 || grid.y < 1 || grid.z < 1) {
    std::fprintf(stderr, "emu: invalid launch grid (%u,%u,%u) block %d lds %zu\n", grid.x, grid.y, grid.z, n,
                 lds_bytes);
    g_last = hipErrorInvalidValue;
    return;
  }
  enqueue(s, [=]() { run_grid(grid, block, lds_bytes, body); });
}

void run_grid(dim3 grid, dim3 block, size_t lds_bytes, const std::function<void()>& body) {
  const int n = (int)(block.x * block.y * block.z);
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) {
        // uninitialised LDS reads as NaN; bytes beyond the launch's size are poisoned
        std::memset(fm::smem, 0xff, lds_bytes);
        ASAN_POISON_MEMORY_REGION(fm::smem + lds_bytes, fm::kEmuLds - lds_bytes);
        const int nw = (n + 63) / 64;
        std::vector<std::unique_ptr<WaveBar>> waves;
        for (int w = 0; w < nw; ++w) waves.emplace_back(new WaveBar(std::min(64, n - 64 * w)));
        BlockBar wg(n, UnparkWaves{&waves});
        g_pool.run(Pool::Block{&body, grid, block, dim3(bx, by, bz), &wg, &waves}, n);
        ASAN_UNPOISON_MEMORY_REGION(fm::smem + lds_bytes, fm::kEmuLds - lds_bytes);
      }
}
}  // namespace emu

void __syncthreads() {
  t_wave->park();
  t_block->arrive_and_wait();
}
void __builtin_amdgcn_wave_barrier() { t_wave->wait(); }
void __builtin_amdgcn_fence(int, const char*) { std::atomic_thread_fence(std::memory_order_seq_cst); }
void sincospi(double x, double* s, double* c) {
  *s = std::sin(M_PI * x);
  *c = std::cos(M_PI * x);
}
void sincospif(float x, float* s, float* c) {
  *s = (float)std::sin(M_PI * (double)x);
  *c = (float)std::cos(M_PI * (double)x);
}

hipError_t hipMalloc(void** p, size_t bytes) {
  *p = std::malloc(bytes ? bytes : 1);
  if (!*p) return hipErrorOutOfMemory;
  std::memset(*p, 0xff, bytes);  // fresh device memory reads as NaN
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  drain_all();  // hipFree waits for the device
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
  *p = std::malloc(bytes ? bytes : 1);
  if (!*p) return hipErrorOutOfMemory;
  std::lock_guard<std::recursive_mutex> lock(g_launch);
  g_pinned[static_cast<const char*>(*p)] = bytes;
  return hipSuccess;
}
hipError_t hipHostFree(void* p) {
  drain_all();
  {
    std::lock_guard<std::recursive_mutex> lock(g_launch);
    g_pinned.erase(static_cast<const char*>(p));
  }
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  drain_all();
  if (bytes) std::memmove(dst, src, bytes);
  return hipSuccess;
}
// true if p lies in a pinned allocation
bool pinned(const void* p) {
  std::lock_guard<std::recursive_mutex> lock(g_launch);
  const char* c = static_cast<const char*>(p);
  auto it = g_pinned.upper_bound(c);
  if (it == g_pinned.begin()) return false;
  --it;
  return c < it->first + it->second;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind k, hipStream_t s) {
  if (k == hipMemcpyHostToDevice && !pinned(src)) {
    // pageable source: consumed before the call returns, after the stream's earlier work
    EmuStream* st = str(s);
    drain([st] { return st->q.empty(); });
    if (bytes) std::memmove(dst, src, bytes);
    return hipSuccess;
  }
  enqueue(s, [=]() {
    if (bytes) std::memmove(dst, src, bytes);
  });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t s) {
  enqueue(s, [=]() {
    if (bytes) std::memset(dst, value, bytes);
  });
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags) {
  std::lock_guard<std::recursive_mutex> lock(g_launch);
  *s = new EmuStream{flags, {}};
  g_streams.push_back(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  drain_all();
  std::lock_guard<std::recursive_mutex> lock(g_launch);
  g_streams.erase(std::find(g_streams.begin(), g_streams.end(), s));
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  EmuStream* st = str(s);
  if (!drain([st] { return st->q.empty(); })) drain_all();
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  std::lock_guard<std::recursive_mutex> lock(g_launch);
  if (!e->done) str(s)->q.push_back({nullptr, e});
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags) {
  *e = new EmuEvent{flags};
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  drain_all();
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lock(g_launch);
  e->done = false;
  ++e->pending;
  str(s)->q.push_back({[e]() {
                         if (--e->pending == 0) e->done = true;
                       },
                       nullptr});
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  if (!drain([e] { return e->done; })) drain_all();
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  // the device makes progress while the host polls
  if (!e->done) drain([e] { return e->done; });
  return e->done ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.001f;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() {
  drain_all();
  return hipSuccess;
}
hipError_t hipGetDevice(int* dev) {
  *dev = 0;
  return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int) {
  std::memset(prop, 0, sizeof(*prop));
  std::snprintf(prop->name, sizeof(prop->name), "cpu-emulation");
  std::snprintf(prop->gcnArchName, sizeof(prop->gcnArchName), "gfx950");
  prop->multiProcessorCount = kEmuCUs;
  prop->totalGlobalMem = (size_t)8 << 30;
  prop->sharedMemPerBlock = fm::kEmuLds;
  prop->warpSize = 64;
  prop->maxThreadsPerBlock = 1024;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* value, hipDeviceAttribute_t, int) {
  *value = kEmuCUs;
  return hipSuccess;
}
hipError_t hipGetLastError() {
  const hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated error"; }
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol) {
  *ptr = const_cast<void*>(symbol);
  return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
