// Host-only stand-in for the HIP runtime, for checking the memory accesses
// of the library's kernels on the CPU under AddressSanitizer: a launch runs
// every thread of every workgroup to completion, one after another.
// Barriers, cross-lane reads and matrix-core instructions become no-ops or
// scalar stand-ins, so values are meaningless; addresses are exact because
// no kernel computes an address from data.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <type_traits>
using std::sqrt; using std::fabs; using std::fma; using std::isinf; using std::isnan;
using std::min; using std::max;
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __shared__ static
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
// a device array's host address stands in for its device address
#define HIP_SYMBOL(sym) (sym)
template <typename T>
inline int hipGetSymbolAddress(void** p, T& sym) {
  *p = (void*)&sym;
  return 0;
}
inline unsigned long long __umul64hi(unsigned long long a, unsigned long long b) {
  return (unsigned long long)(((unsigned __int128)a * b) >> 64);
}
struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
inline dim3 threadIdx, blockIdx, blockDim, gridDim;
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorInvalidDevice = 101 };
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice, hipMemcpyDeviceToHost,
                     hipMemcpyDeviceToDevice, hipMemcpyDefault };
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  memcpy(d, s, n);
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline void __syncthreads() {}
inline void __threadfence() {}
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) ((c) + (a) * (b))
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) ((c) + (a) * (b))
#define __builtin_amdgcn_readlane(v, l) (v)
#define __builtin_amdgcn_ds_bpermute(addr, v) (v)
#define __builtin_amdgcn_update_dpp(old, v, ctrl, rm, bm, bc) (v)
#define __builtin_amdgcn_mov_dpp(v, ctrl, rm, bm, bc) (v)
#define __builtin_amdgcn_readfirstlane(v) (v)
typedef unsigned emu_u32x2 __attribute__((ext_vector_type(2)));
struct double2 {
  double x, y;
};
inline emu_u32x2 __builtin_amdgcn_permlane16_swap(unsigned a, unsigned b, bool, bool) { return emu_u32x2{a, b}; }
inline emu_u32x2 __builtin_amdgcn_permlane32_swap(unsigned a, unsigned b, bool, bool) { return emu_u32x2{a, b}; }
inline int atomicMin(int* p, int v) { const int o = *p; if (v < o) *p = v; return o; }
// GPU inline assembly has no host meaning: it leaves its operands as they are.
#define asm(...) ((void)0)
#define BD_ASM(...) ((void)0)
#define __builtin_amdgcn_rsq(d) (1.0 / std::sqrt(d))
#define __builtin_amdgcn_rcp(d) (1.0 / (d))
#define __builtin_amdgcn_fence(...) ((void)0)
#define __builtin_amdgcn_wave_barrier() ((void)0)
#define __builtin_amdgcn_sched_barrier(m) ((void)0)
#define __builtin_amdgcn_sched_group_barrier(m, n, i) ((void)0)
// Load to LDS: each lane's `size` bytes from its global address land at
// the wave-uniform LDS address plus offset plus lane * size.
inline void __builtin_amdgcn_global_load_lds(const void* src, void* lds, unsigned size, int offset, int) {
  memcpy(static_cast<char*>(lds) + offset + (threadIdx.x & 63) * size, src, size);
}
#define __builtin_amdgcn_s_barrier() ((void)0)
#define __builtin_amdgcn_s_setprio(p) ((void)0)
#define __builtin_amdgcn_s_sleep(n) ((void)0)
#define __builtin_amdgcn_s_waitcnt(n) ((void)0)
#define __noinline__ __attribute__((noinline))
#define __HIP_MEMORY_SCOPE_AGENT 3
// launches run one thread at a time: plain accesses stand in for atomics
template <typename T> inline T emu_atomic_load(T* p) { return *p; }
template <typename T, typename V> inline void emu_atomic_store(T* p, V v) { *p = (T)v; }
template <typename T, typename V> inline T emu_atomic_fetch_add(T* p, V v) { const T o = *p; *p = o + (T)v; return o; }
#define __hip_atomic_load(p, o, s) emu_atomic_load(p)
#define __hip_atomic_store(p, v, o, s) emu_atomic_store((p), (v))
#define __hip_atomic_fetch_add(p, v, o, s) emu_atomic_fetch_add((p), (v))
template <typename T> inline T __shfl_xor(T v, int, int = 64) { return v; }
extern long g_emu_launches;
// Optional observer of every launch: kernel address, grid, and the
// arguments as 64-bit values (pointers as addresses, integers as values,
// anything else as 0).
typedef void (*emu_observer_t)(const void* kernel, dim3 grid, const int64_t* args, int nargs);
inline emu_observer_t g_emu_observer = nullptr;
// A kernel whose threads are not run (only observed), e.g. one too large to
// emulate at a given size.
inline const void* g_emu_skip = nullptr;
template <typename T>
inline int64_t emu_arg(T v) {
  if constexpr (std::is_pointer_v<T>) return (int64_t)(uintptr_t)v;
  else if constexpr (std::is_integral_v<T> || std::is_enum_v<T>) return (int64_t)v;
  else return 0;
}
template <typename K, typename... Args>
inline void emu_launch(K kernel, dim3 grid, dim3 block, Args... args) {
  ++g_emu_launches;
  if (g_emu_observer) {
    const int64_t a[] = {emu_arg(args)..., 0};
    g_emu_observer((const void*)kernel, grid, a, (int)sizeof...(Args));
  }
  if ((const void*)kernel == g_emu_skip) return;
  gridDim = grid;
  blockDim = block;
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx)
        for (unsigned tz = 0; tz < block.z; ++tz)
          for (unsigned ty = 0; ty < block.y; ++ty)
            for (unsigned tx = 0; tx < block.x; ++tx) {
              blockIdx = dim3(bx, by, bz);
              threadIdx = dim3(tx, ty, tz);
              kernel(args...);
            }
}
#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) emu_launch(kernel, dim3(grid), dim3(block), __VA_ARGS__)
