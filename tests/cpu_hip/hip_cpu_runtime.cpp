// CPU implementation of tests/cpu_hip/hip/hip_runtime.h (test infrastructure).
#include "hip/hip_runtime.h"

#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <vector>

thread_local hip_cpu_index threadIdx, blockIdx, blockDim, gridDim;

namespace {

// Barrier over the live threads of the running block: a thread that has
// returned from the kernel no longer takes part.
struct BlockSync {
  std::mutex mu;
  std::condition_variable cv;
  int live = 0, arrived = 0;
  long generation = 0;
  std::vector<double> lanes;   // __shfl_xor exchange, one slot per thread

  void arrive_and_wait() {
    std::unique_lock<std::mutex> lk(mu);
    const long gen = generation;
    if (++arrived == live) {
      arrived = 0;
      ++generation;
      cv.notify_all();
      return;
    }
    cv.wait(lk, [&] { return generation != gen; });
  }
  void leave() {
    std::lock_guard<std::mutex> lk(mu);
    --live;
    if (live > 0 && arrived == live) {
      arrived = 0;
      ++generation;
      cv.notify_all();
    }
  }
};

BlockSync* g_block = nullptr;

unsigned flat_tid() { return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z); }

}  // namespace

void __syncthreads() { g_block->arrive_and_wait(); }

int atomicOr(int* p, int v) {
  std::lock_guard<std::mutex> lk(g_block->mu);
  const int old = *p;
  *p = old | v;
  return old;
}

// Called by every thread of the block together (as the kernels here do).
double __shfl_xor(double v, int lane_mask, int width) {
  const unsigned t = flat_tid();
  const unsigned base = t - t % (unsigned)width;
  g_block->lanes[t] = v;
  g_block->arrive_and_wait();
  const double r = g_block->lanes[base + ((t - base) ^ (unsigned)lane_mask)];
  g_block->arrive_and_wait();
  return r;
}

namespace {

// Persistent worker threads (one per thread of the largest block so far):
// each launch hands the block's threads to the first nt workers.
struct Pool {
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_job, cv_done;
  long gen = 0;
  unsigned njobs = 0, acked = 0;
  const std::function<void(unsigned)>* job = nullptr;
  bool quit = false;

  // called with mu held: a new worker starts at the current generation, so
  // it waits for the next job instead of taking the last one
  void ensure(unsigned n) {
    while (workers.size() < n) {
      const unsigned id = (unsigned)workers.size();
      const long start = gen;
      workers.emplace_back([this, id, start] {
        long seen = start;
        for (;;) {
          const std::function<void(unsigned)>* fn;
          unsigned nj;
          {
            std::unique_lock<std::mutex> lk(mu);
            cv_job.wait(lk, [&] { return quit || gen != seen; });
            if (quit) return;
            seen = gen;
            fn = job;
            nj = njobs;
          }
          if (id < nj) (*fn)(id);
          std::lock_guard<std::mutex> lk(mu);
          if (++acked == workers.size()) cv_done.notify_all();
        }
      });
    }
  }
  void run(unsigned n, const std::function<void(unsigned)>& fn) {
    std::unique_lock<std::mutex> lk(mu);
    ensure(n);
    job = &fn;
    njobs = n;
    acked = 0;
    ++gen;
    cv_job.notify_all();
    cv_done.wait(lk, [&] { return acked == workers.size(); });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(mu);
      quit = true;
    }
    cv_job.notify_all();
    for (auto& w : workers) w.join();
  }
};

Pool& pool() {
  static Pool p;
  return p;
}

}  // namespace

void hip_cpu_launch(const std::function<void()>& body, dim3 grid, dim3 block) {
  const unsigned nt = block.x * block.y * block.z;
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) {
        BlockSync sync;
        sync.live = (int)nt;
        sync.lanes.assign(nt, 0.0);
        g_block = &sync;
        const std::function<void(unsigned)> fn = [&](unsigned t) {
          threadIdx = {t % block.x, (t / block.x) % block.y, t / (block.x * block.y)};
          blockIdx = {bx, by, bz};
          blockDim = {block.x, block.y, block.z};
          gridDim = {grid.x, grid.y, grid.z};
          body();
          sync.leave();
        };
        pool().run(nt, fn);
        g_block = nullptr;
      }
}

hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipGetDevice(int* dev) {
  *dev = 0;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "error"; }
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
  std::memmove(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }

struct hip_cpu_event {
  int dummy;
};
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new hip_cpu_event{0};
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.0f;
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
