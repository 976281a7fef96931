// Host-only stand-in for the HIP runtime header, for building the library's host code
// (api.hip, server.hip) with g++ and the thread / address sanitizers on a machine without
// a GPU.  Device memory is host memory; each stream is a worker thread that runs the
// enqueued copies and stub kernels in order (stub_runtime.cpp, stub_kernels.cpp).
#pragma once

#include <stddef.h>
#include <stdint.h>

#define __host__
#define __device__
#define __global__
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (&(x))

typedef enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotReady = 600
} hipError_t;

typedef enum {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum {
  hipDeviceAttributeMultiprocessorCount = 0,
  hipDeviceAttributeWallClockRate = 1
} hipDeviceAttribute_t;

#define hipStreamNonBlocking 1u
#define hipHostMallocDefault 0u

struct ihipStream_t;
typedef ihipStream_t* hipStream_t;
struct ihipEvent_t;
typedef ihipEvent_t* hipEvent_t;

hipError_t hipGetDeviceCount(int* count);
hipError_t hipSetDevice(int device);
hipError_t hipDeviceGetAttribute(int* value, hipDeviceAttribute_t attr, int device);
hipError_t hipGetLastError(void);
hipError_t hipMalloc(void** ptr, size_t bytes);
hipError_t hipFree(void* ptr);
hipError_t hipHostMalloc(void** ptr, size_t bytes, unsigned int flags);
hipError_t hipHostFree(void* ptr);
hipError_t hipMemGetInfo(size_t* free_bytes, size_t* total_bytes);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipEventSynchronize(hipEvent_t e);

// Graphs: a stream in capture records its tasks instead of running them; a launched graph
// enqueues the recorded tasks on the target stream.
typedef enum { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1, hipStreamCaptureModeRelaxed = 2 }
    hipStreamCaptureMode;
struct ihipGraph_t;
typedef ihipGraph_t* hipGraph_t;
struct ihipGraphExec_t;
typedef ihipGraphExec_t* hipGraphExec_t;
struct hipGraphNode;
typedef hipGraphNode* hipGraphNode_t;
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* err_node, char* log, size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphDestroy(hipGraph_t g);
