// CPU emulation of the part of the HIP runtime and device language that the library
// uses, for a host build of the device code (g++, with AddressSanitizer and
// UndefinedBehaviorSanitizer).  Test infrastructure only.
//
// * Device memory is host memory from malloc, so the sanitizer checks every global
//   access against its allocation.
// * A launch runs every workgroup of the grid, one after the other, each as blockDim
//   host threads; __syncthreads is a barrier over the workgroup's live threads, the
//   wavefront barrier one over the live threads of its 64-lane wavefront, and a thread
//   that returns leaves both.  Dynamic LDS is one static array whose bytes beyond the
//   launch's dynamic size are poisoned for the sanitizer during the launch.
// * Streams are queues: launches, memsets and copies from pinned host memory
//   (hipHostMalloc) are enqueued and run only when the host synchronises (stream, event
//   or device), in an order that takes the most recently created runnable stream first
//   and honours hipStreamWaitEvent, so that a host buffer reused, or memory freed, before
//   the work that reads it has run shows up as wrong data or a sanitizer report.  Copies
//   from pageable memory wait for the stream and complete before returning, as HIP's do.
// * The device reports few compute units, so persistent grids loop over many tiles.
#pragma once
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <functional>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...)
#define __shared__
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (reinterpret_cast<const void*>(&(x)))
// occupancy hints of the kernels mean nothing here (the attribute list becomes empty)
#define amdgpu_waves_per_eu(...)

// the device library's min / max over mixed arithmetic types
template <class A, class B>
inline auto min(A a, B b) -> decltype(a + b) {
  return a < b ? a : b;
}
template <class A, class B>
inline auto max(A a, B b) -> decltype(a + b) {
  return a < b ? b : a;
}

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct EmuIdx {
  unsigned x, y, z;
};
extern thread_local EmuIdx threadIdx, blockIdx, blockDim, gridDim;

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotReady = 600,
  hipErrorNotSupported = 801,
  hipErrorLaunchFailure = 719,
} hipError_t;

typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4,
} hipMemcpyKind;

typedef enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1 } hipDeviceAttribute_t;
typedef enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 } hipFuncAttribute;

struct EmuStream;
struct EmuEvent;
typedef EmuStream* hipStream_t;
typedef EmuEvent* hipEvent_t;

struct hipDeviceProp_t {
  char name[256];
  char gcnArchName[256];
  int multiProcessorCount;
  size_t totalGlobalMem;
  size_t sharedMemPerBlock;
  int warpSize;
  int maxThreadsPerBlock;
};

#define hipStreamNonBlocking 1
#define hipEventDisableTiming 2
#define hipHostMallocDefault 0

hipError_t hipMalloc(void** p, size_t bytes);
template <typename T>
hipError_t hipMalloc(T** p, size_t bytes) {
  return hipMalloc(reinterpret_cast<void**>(p), bytes);
}
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
template <typename T>
hipError_t hipHostMalloc(T** p, size_t bytes, unsigned flags = 0) {
  return hipHostMalloc(reinterpret_cast<void**>(p), bytes, flags);
}
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s = nullptr);
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t s = nullptr);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipDeviceSynchronize();
hipError_t hipGetDevice(int* dev);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int dev);
hipError_t hipDeviceGetAttribute(int* value, hipDeviceAttribute_t attr, int dev);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol);
hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute attr, int value);
template <typename F>
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, F, int, size_t) {
  *n = 2;
  return hipSuccess;
}

// device intrinsics
void __syncthreads();
void __builtin_amdgcn_wave_barrier();
void __builtin_amdgcn_fence(int order, const char* scope);
void sincospi(double x, double* s, double* c);
void sincospif(float x, float* s, float* c);

namespace emu {
// a kernel launch enqueued on a stream (arguments captured by value, run when the
// stream's work is executed)
void launch(hipStream_t s, dim3 grid, dim3 block, size_t lds_bytes, std::function<void()> body);
}  // namespace emu

#define hipLaunchKernelGGL(kern, grid, block, lds, stream, ...) \
  ::emu::launch((stream), (grid), (block), (lds), [=]() { (kern)(__VA_ARGS__); })
