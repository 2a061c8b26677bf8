// Host-only stand-in for the HIP runtime, used to build the library's host
// code (graph upload, pass driver, server scheduler) on a machine without a
// GPU so its threading and memory logic can run under AddressSanitizer and
// ThreadSanitizer.  "Device" memory is host memory; the few grid-stride
// kernels defined in host translation units run sequentially on the CPU.
// Test infrastructure only: nothing in the product includes this file.
#pragma once
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __align__(x) alignas(x)

struct dim3 {
    uint32_t x, y, z;
    dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};
struct uint2 {
    uint32_t x, y;
};
inline uint2 make_uint2(uint32_t a, uint32_t b) { return uint2{a, b}; }
struct uint4 {
    uint32_t x, y, z, w;
};
inline uint4 make_uint4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) { return uint4{a, b, c, d}; }

extern thread_local dim3 blockIdx, threadIdx, blockDim, gridDim;

typedef enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 } hipError_t;
typedef enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 } hipMemcpyKind;
typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
typedef struct ihipGraphExec_t *hipGraphExec_t;
struct hipDeviceProp_t {
    int multiProcessorCount;
};
#define hipStreamNonBlocking 1
#define hipHostMallocDefault 0
#define HIP_SYMBOL(x) (&(x))

namespace hipsim {
extern std::mutex launch_mu;  // one simulated kernel at a time
template <typename F, typename... A>
void launch(F f, dim3 g, dim3 b, A... a) {
    std::lock_guard<std::mutex> lk(launch_mu);
    gridDim = g;
    blockDim = b;
    for (uint32_t bx = 0; bx < g.x; bx++)
        for (uint32_t tx = 0; tx < b.x; tx++) {
            blockIdx = dim3(bx, 0, 0);
            threadIdx = dim3(tx, 0, 0);
            f(a...);
        }
}
}  // namespace hipsim

#define hipLaunchKernelGGL(kernel, grid, block, shm, stream, ...) \
    ::hipsim::launch(kernel, dim3(grid), dim3(block), __VA_ARGS__)

template <typename T>
inline T atomicOr(T *p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
template <typename T>
inline T atomicAdd(T *p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }

hipError_t hipSetDevice(int);
hipError_t hipGetDevice(int *);
hipError_t hipGetDeviceProperties(hipDeviceProp_t *, int);
hipError_t hipMalloc(void **, size_t);
hipError_t hipFree(void *);
hipError_t hipHostMalloc(void **, size_t, unsigned);
hipError_t hipHostFree(void *);
hipError_t hipMemcpyAsync(void *, const void *, size_t, hipMemcpyKind, hipStream_t);
hipError_t hipMemsetAsync(void *, int, size_t, hipStream_t);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipStreamCreateWithFlags(hipStream_t *, unsigned);
hipError_t hipStreamDestroy(hipStream_t);
hipError_t hipEventCreate(hipEvent_t *);
hipError_t hipEventRecord(hipEvent_t, hipStream_t);
hipError_t hipEventSynchronize(hipEvent_t);
hipError_t hipEventElapsedTime(float *, hipEvent_t, hipEvent_t);
hipError_t hipEventDestroy(hipEvent_t);
hipError_t hipGetLastError();
hipError_t hipGetSymbolAddress(void **, const void *);
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t);
hipError_t hipGraphExecDestroy(hipGraphExec_t);
const char *hipGetErrorString(hipError_t);
