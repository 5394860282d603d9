// CPU emulation of the subset of HIP used by the library, for tests only:
// the library's kernels and host code compiled with a host compiler, a
// pool of host threads standing in for the threads of a block, a barrier for
// __syncthreads, host memory standing in for device memory.  Built with AddressSanitizer it
// reports any out-of-bounds access of a kernel with a stack trace.
#pragma once
#include <atomic>
#include <barrier>
#include <condition_variable>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (&(x))
#define HIP_DYNAMIC_SHARED(type, var) type* var = reinterpret_cast<type*>(emu::dyn_shared());

struct dim3 {
  unsigned x = 1, y = 1, z = 1;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorNotReady = 600, hipErrorInvalidValue = 1 };
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice,
                     hipMemcpyDefault };
enum { hipStreamNonBlocking = 1, hipHostMallocDefault = 0, hipEventDisableTiming = 2 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };

namespace emu {
struct Graph {
  std::vector<std::function<void()>> ops;
};
struct Stream {
  Graph* capture = nullptr;
};
struct Event {};
struct Ctx {
  dim3 tid, bid, bdim, gdim;
};
inline thread_local Ctx ctx;
inline std::barrier<>* g_bar = nullptr;
inline std::vector<char> g_dyn;
inline std::vector<double> g_shfl;
inline std::mutex g_atomic_mu;
inline char* dyn_shared() { return g_dyn.data(); }

// A pool of host threads, created once and grown to the largest block seen,
// runs the blocks of every launch one after the other: thread t plays GPU
// thread t of the current block.  A fresh barrier per block lets threads that
// leave the kernel early drop out of later __syncthreads, as exited waves do
// on the device.
struct Pool {
  std::mutex mu;
  std::condition_variable cv_go, cv_done;
  uint64_t gen = 0;
  unsigned remaining = 0;
  const std::function<void()>* fn = nullptr;
  dim3 grid, block, bid;
  std::vector<std::thread> th;
  bool stop = false;

  void worker(unsigned t) {
    uint64_t seen = 0;
    for (;;) {
      std::unique_lock<std::mutex> lk(mu);
      cv_go.wait(lk, [&] { return gen != seen || stop; });
      if (stop) return;
      seen = gen;
      if (t >= block.x) continue;
      ctx.tid = dim3(t);
      ctx.bid = bid;
      ctx.bdim = block;
      ctx.gdim = grid;
      const std::function<void()>* f = fn;
      lk.unlock();
      (*f)();
      g_bar->arrive_and_drop();
      lk.lock();
      if (--remaining == 0) cv_done.notify_one();
    }
  }
  void run_block(const std::function<void()>& f, dim3 g, dim3 b, unsigned blk) {
    std::unique_lock<std::mutex> lk(mu);
    while (th.size() < b.x) {
      const unsigned t = (unsigned)th.size();
      th.emplace_back([this, t] { worker(t); });
    }
    fn = &f;
    grid = g;
    block = b;
    bid = dim3(blk);
    remaining = b.x;
    ++gen;
    cv_go.notify_all();
    cv_done.wait(lk, [&] { return remaining == 0; });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv_go.notify_all();
    for (auto& x : th) x.join();
  }
};
inline Pool g_pool;

inline std::mutex g_launch_mu;  // one launch at a time, whatever host thread issues it

inline void run_kernel(dim3 grid, dim3 block, size_t shmem, const std::function<void()>& fn) {
  std::lock_guard<std::mutex> lk(g_launch_mu);
  for (unsigned b = 0; b < grid.x; ++b) {
    std::barrier<> bar((std::ptrdiff_t)block.x);
    g_bar = &bar;
    g_dyn.assign(shmem + 64, 0);
    g_shfl.assign(block.x, 0.0);
    g_pool.run_block(fn, grid, block, b);
    g_bar = nullptr;
  }
}

inline void launch(void* stream, dim3 grid, dim3 block, size_t shmem, std::function<void()> fn) {
  Stream* s = reinterpret_cast<Stream*>(stream);
  if (s && s->capture) {
    s->capture->ops.push_back([=] { run_kernel(grid, block, shmem, fn); });
    return;
  }
  run_kernel(grid, block, shmem, fn);
}
}  // namespace emu

typedef emu::Stream* hipStream_t;
typedef emu::Event* hipEvent_t;
typedef emu::Graph* hipGraph_t;
typedef emu::Graph* hipGraphExec_t;

#define threadIdx (emu::ctx.tid)
#define blockIdx (emu::ctx.bid)
#define blockDim (emu::ctx.bdim)
#define gridDim (emu::ctx.gdim)

inline void __syncthreads() { emu::g_bar->arrive_and_wait(); }

template <typename T>
inline T atomicAdd(T* p, T v) {
  std::lock_guard<std::mutex> lk(emu::g_atomic_mu);
  T o = *p;
  *p = o + v;
  return o;
}
template <typename T>
inline void unsafeAtomicAdd(T* p, T v) {
  atomicAdd(p, v);
}

// lane exchange inside a block through block scratch: every thread of the
// block must take part (two barriers per call)
template <typename T>
inline T __shfl_xor(T v, int mask, int w = 64) {
  const unsigned t = threadIdx.x;
  emu::g_shfl[t] = (double)v;
  __syncthreads();
  const unsigned o = t ^ (unsigned)mask;
  const double r = (o < blockDim.x && (o / (unsigned)w) == (t / (unsigned)w)) ? emu::g_shfl[o] : (double)v;
  __syncthreads();
  return (T)r;
}

// data-parallel lane moves used by the kernels (gfx9 DPP controls: quad
// permutation 0x00-0xFF, row half mirror 0x141), through block scratch:
// every thread of the block must take part
// scheduling barrier of the device compiler: nothing to do on the host
inline void __builtin_amdgcn_sched_barrier(int) {}
// a wavefront-wide barrier: the lanes of the emulated block (the kernels use
// it only in one-wavefront blocks) meet here, as the hardware wave executes
// them in lockstep
inline void __builtin_amdgcn_wave_barrier() { __syncthreads(); }
inline void __builtin_amdgcn_fence(int, const char*) {}
inline int __builtin_amdgcn_mov_dpp(int v, int ctrl, int, int, bool) {
  const unsigned t = threadIdx.x;
  emu::g_shfl[t] = (double)v;
  __syncthreads();
  unsigned src = t;
  if (ctrl >= 0 && ctrl <= 0xFF) {
    src = (t & ~3u) + ((unsigned)(ctrl >> (2 * (t & 3))) & 3u);
  } else if (ctrl == 0x141) {
    src = (t & ~7u) + (7u - (t & 7u));
  } else {
    std::abort();
  }
  const int r = src < blockDim.x ? (int)emu::g_shfl[src] : v;
  __syncthreads();
  return r;
}
inline float __int_as_float(int v) {
  float f;
  std::memcpy(&f, &v, 4);
  return f;
}
inline int __float_as_int(float f) {
  int v;
  std::memcpy(&v, &f, 4);
  return v;
}
inline double __longlong_as_double(long long v) {
  double d;
  std::memcpy(&d, &v, 8);
  return d;
}
inline long long __double_as_longlong(double d) {
  long long v;
  std::memcpy(&v, &d, 8);
  return v;
}

// wave-wide shuffle through block scratch (waves of 64 lanes)
inline double __shfl_down(double v, int o, int w) {
  const unsigned t = threadIdx.x, lane = t % (unsigned)w;
  emu::g_shfl[t] = v;
  __syncthreads();
  double r = (lane + (unsigned)o < (unsigned)w && t + (unsigned)o < blockDim.x) ? emu::g_shfl[t + o] : v;
  __syncthreads();
  return r;
}

namespace emu {
// kernel arguments are evaluated and copied at the launch, as on the device
template <typename F, typename... A>
inline void launch_k(void* stream, dim3 grid, dim3 block, size_t shmem, F* kernel, A... args) {
  launch(stream, grid, block, shmem, [=]() { kernel(args...); });
}
}  // namespace emu

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  emu::launch_k((void*)(stream), dim3(grid), dim3(block), (size_t)(shmem), kernel, __VA_ARGS__)

inline const char* hipGetErrorString(hipError_t) { return "emulated HIP error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  std::memcpy(dst, src, n);
  return hipSuccess;
}
inline hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t) {
  std::memset(dst, v, n);
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new emu::Stream();
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
inline hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new emu::Event();
  return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new emu::Event();
  return hipSuccess;
}
// device memory is host memory here: a device variable's address is its own
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
// launches run when issued, so every recorded event has completed
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.0f;
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
  *p = std::calloc(1, n);
  return hipSuccess;
}
inline hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}
inline hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  s->capture = new emu::Graph();
  return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  *g = s->capture;
  s->capture = nullptr;
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t) {
  *e = new emu::Graph(*g);
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto& op : e->ops) op();
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
