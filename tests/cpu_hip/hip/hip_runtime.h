// CPU stand-in for the part of the HIP runtime the library's kernels and
// host code use, so the same sources build with g++ for the host (test
// infrastructure only: tests/test_cpu_kernels.py builds the library this
// way under AddressSanitizer and checks it against the oracle).  A kernel
// launch runs its blocks one after another; each block runs one OS thread
// per GPU thread, __syncthreads is a barrier over the block's live threads,
// and __shared__ variables are function statics (one block at a time).
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <functional>

using std::isfinite;

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __shared__ static
#define __launch_bounds__(...)
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (&(x))
#define __restrict__ __restrict
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))
#define __builtin_nontemporal_load(p) (*(p))
#define __builtin_nontemporal_store(v, p) (*(p) = (v))

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint4 {
  unsigned x, y, z, w;
};
struct hip_cpu_index {
  unsigned x, y, z;
};
extern thread_local hip_cpu_index threadIdx, blockIdx, blockDim, gridDim;

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorNotReady = 2 };
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
typedef void* hipStream_t;
typedef struct hip_cpu_event* hipEvent_t;

void __syncthreads();
int atomicOr(int* p, int v);
double __shfl_xor(double v, int lane_mask, int width = 64);

void hip_cpu_launch(const std::function<void()>& body, dim3 grid, dim3 block);
#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  hip_cpu_launch([&]() { kernel(__VA_ARGS__); }, dim3(grid), dim3(block))

hipError_t hipGetLastError();
hipError_t hipGetDevice(int* dev);
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
const char* hipGetErrorString(hipError_t e);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipEventDestroy(hipEvent_t e);
