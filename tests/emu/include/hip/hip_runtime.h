// Host emulation of the parts of the HIP runtime and device language the
// MCG library uses, for a plain C++20 build of the library (kernels and
// driver) that runs on the CPU under AddressSanitizer.  Test
// infrastructure only: the product is built with hipcc for gfx950.
//
// Device memory is host memory (malloc).  A kernel launch runs every block
// in turn; the threads of a block run as std::threads, so __syncthreads is a
// real barrier and __shfl_xor a real exchange between the lanes of a
// 64-wide wave.  Streams are synchronous.  Stream capture records launches
// and memory operations; a graph launch replays them.
#pragma once

#include <algorithm>
#include <barrier>
#include <condition_variable>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <semaphore>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (&(x))
#define __shared__ static thread_local_block_shared

using std::atan2;
using std::fabs;
using std::fmin;
using std::sqrt;

struct float2 {
  float x, y;
};
struct double2 {
  double x, y;
};
inline double2 make_double2(double a, double b) { return double2{a, b}; }
inline float2 make_float2(float a, float b) { return float2{a, b}; }

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace emu {
struct BlockCtx {
  std::barrier<> *bar;
  std::vector<unsigned char> *slots;  // 8 bytes per lane
};
inline thread_local dim3 t_block, t_thread, t_bdim, t_gdim;
inline thread_local BlockCtx t_ctx{nullptr, nullptr};
inline std::mutex &atomic_mutex() {
  static std::mutex m;
  return m;
}
}  // namespace emu

#define blockIdx (emu::t_block)
#define threadIdx (emu::t_thread)
#define blockDim (emu::t_bdim)
#define gridDim (emu::t_gdim)
// __shared__ arrays are only declared inside device functions; blocks run one
// at a time, so a plain static works (all lanes of the block share it)
#define thread_local_block_shared

inline void __syncthreads() { emu::t_ctx.bar->arrive_and_wait(); }

template <typename T> inline T __shfl_xor(T v, int mask, int width = 64) {
  static_assert(sizeof(T) <= 8, "shuffle of at most 8 bytes");
  const unsigned lane = emu::t_thread.x;
  unsigned char *s = emu::t_ctx.slots->data();
  std::memcpy(s + 8 * lane, &v, sizeof(T));
  emu::t_ctx.bar->arrive_and_wait();
  const unsigned src = ((lane % width) ^ (unsigned)mask) + (lane / width) * width;
  T r;
  std::memcpy(&r, s + 8 * src, sizeof(T));
  emu::t_ctx.bar->arrive_and_wait();
  return r;
}

inline int atomicOr(int *p, int v) {
  std::lock_guard<std::mutex> g(emu::atomic_mutex());
  int o = *p;
  *p = o | v;
  return o;
}
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v) {
  std::lock_guard<std::mutex> g(emu::atomic_mutex());
  unsigned long long o = *p;
  *p = o + v;
  return o;
}

// ------------------------------------------------------------------ runtime
enum hipError_t { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
#define hipStreamNonBlocking 1
#define hipHostMallocDefault 0

struct emu_stream {
  int id;
};
typedef emu_stream *hipStream_t;
struct emu_event {
  double t;
};
typedef emu_event *hipEvent_t;
struct emu_graph {
  std::vector<std::function<void()>> ops;
};
typedef emu_graph *hipGraph_t;
typedef emu_graph *hipGraphExec_t;

namespace emu {
inline hipStream_t &capturing() {
  static hipStream_t s = nullptr;
  return s;
}
inline emu_graph *&capture_graph() {
  static emu_graph *g = nullptr;
  return g;
}
// run now, or record when the stream is being captured
inline void submit(hipStream_t s, std::function<void()> f) {
  if (capturing() && s == capturing())
    capture_graph()->ops.push_back(std::move(f));
  else
    f();
}
// Persistent lane threads: run(n, f) calls f(t) on threads t = 0..n-1 and
// returns when all have finished (threads are created once and reused; each
// waits on its own semaphore, so a launch wakes only the lanes it uses).
class LanePool {
 public:
  static constexpr unsigned MAXLANES = 1024;  // the largest block HIP allows
  static LanePool &get() {
    static LanePool *p = new LanePool;  // never destroyed: idle workers may outlive main
    return *p;
  }
  void run(unsigned n, const std::function<void(unsigned)> &f) {
    if (n > MAXLANES) std::abort();
    {
      std::lock_guard<std::mutex> lk(m_);
      while (nth_ < n) {
        const unsigned id = nth_++;
        sem_[id] = std::make_unique<std::binary_semaphore>(0);
        std::thread([this, id] { work(id); }).detach();
      }
      task_ = &f;
      left_ = n;
    }
    for (unsigned t = 0; t < n; t++) sem_[t]->release();  // publishes task_ to lane t
    std::unique_lock<std::mutex> lk(m_);
    done_.wait(lk, [this] { return left_ == 0; });
    task_ = nullptr;
  }

 private:
  void work(unsigned id) {
    for (;;) {
      sem_[id]->acquire();
      const std::function<void(unsigned)> *f = task_;
      (*f)(id);
      std::lock_guard<std::mutex> lk(m_);
      if (--left_ == 0) done_.notify_one();
    }
  }
  std::mutex m_;
  std::condition_variable done_;
  std::unique_ptr<std::binary_semaphore> sem_[MAXLANES];
  const std::function<void(unsigned)> *task_ = nullptr;
  unsigned nth_ = 0, left_ = 0;
};

template <typename F> void run_grid(dim3 grid, dim3 block, F body) {
  const unsigned nthreads = block.x * block.y * block.z;
  for (unsigned bz = 0; bz < grid.z; bz++)
    for (unsigned by = 0; by < grid.y; by++)
      for (unsigned bx = 0; bx < grid.x; bx++) {
        std::barrier<> bar((std::ptrdiff_t)nthreads);
        std::vector<unsigned char> slots(8 * nthreads);
        const std::function<void(unsigned)> lane = [&](unsigned t) {
          t_block = dim3(bx, by, bz);
          t_thread = dim3(t % block.x, (t / block.x) % block.y, t / (block.x * block.y));
          t_bdim = block;
          t_gdim = grid;
          t_ctx = BlockCtx{&bar, &slots};
          body();
          bar.arrive_and_drop();
        };
        LanePool::get().run(nthreads, lane);
      }
}
}  // namespace emu

// kernel launch: EMU_LAUNCH(kernel, grid, block, stream, args...)
#define EMU_LAUNCH(KERNEL, GRID, BLOCK, STREAM, ...)                              \
  emu::submit((STREAM), [=] { emu::run_grid(dim3(GRID), dim3(BLOCK), [=] { KERNEL(__VA_ARGS__); }); })

inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "success" : "emulated error"; }
inline hipError_t hipGetDeviceCount(int *n) {
  *n = 1;
  return hipSuccess;
}
inline hipError_t hipSetDevice(int) { return hipSuccess; }
// a __device__ variable is a host variable here: its address is the symbol's
inline hipError_t hipGetSymbolAddress(void **p, const void *symbol) {
  *p = const_cast<void *>(symbol);
  return hipSuccess;
}
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipMalloc(void **p, size_t n) {
  *p = std::malloc(n);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void *p) {
  std::free(p);
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
inline hipError_t hipHostFree(void *p) { return hipFree(p); }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t st) {
  emu::submit(st, [=] { std::memcpy(d, s, n); });
  return hipSuccess;
}
inline hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t st) {
  emu::submit(st, [=] { std::memset(d, v, n); });
  return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  static int next = 1;
  *s = new emu_stream{next++};
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
inline hipError_t hipEventCreate(hipEvent_t *e) {
  *e = new emu_event{0.0};
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  e->t = (double)clock() / CLOCKS_PER_SEC * 1000.0;
  return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)std::max(1e-3, b->t - a->t);
  return hipSuccess;
}
inline hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  emu::capturing() = s;
  emu::capture_graph() = new emu_graph();
  return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
  *g = emu::capture_graph();
  emu::capturing() = nullptr;
  emu::capture_graph() = nullptr;
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, void *, char *, size_t) {
  *e = new emu_graph(*g);
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto &op : e->ops) op();
  return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete e;
  return hipSuccess;
}
