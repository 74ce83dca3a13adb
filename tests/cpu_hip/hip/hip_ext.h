// CPU stand-in for <hip/hip_ext.h>: the extended launch runs the kernel like
// hipLaunchKernelGGL; its timing events are not recorded.
#pragma once
#include "hip_runtime.h"

#define hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, start, stop, flags, ...) \
  hip_cpu_launch([&]() { kernel(__VA_ARGS__); }, dim3(grid), dim3(block))
