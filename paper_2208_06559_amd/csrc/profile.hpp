// Optional per-kernel timing with HIP events on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

namespace bd {

struct Profiler;
// Active profiler of the calling thread (set by the C ABI for the duration
// of a call on a handle that has profiling enabled), else null.
extern thread_local Profiler* g_prof;

void prof_mark_begin(hipStream_t s, const char* name);
void prof_mark_end(hipStream_t s);

}  // namespace bd

// Launch with optional start/stop events around the kernel.
#define BD_LAUNCH(name, kernel, grid, block, shmem, stream, ...)                \
  do {                                                                        \
    if (::bd::g_prof) ::bd::prof_mark_begin((stream), (name));                \
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);      \
    if (::bd::g_prof) ::bd::prof_mark_end((stream));                          \
  } while (0)
