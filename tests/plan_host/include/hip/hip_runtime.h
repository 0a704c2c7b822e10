// Host-only model of the HIP runtime calls the plan executor makes (test infrastructure:
// the executor's C++ is compiled with the host compiler and AddressSanitizer against this
// header and hip_model.cpp, no GPU).  Only types and host API declarations.
#pragma once
#include <cstddef>
#include <cstdint>

typedef int hipError_t;
enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorInvalidSymbol = 13,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidResourceHandle = 400,
  hipErrorNotReady = 600,
  hipErrorStreamCaptureUnsupported = 900,
  hipErrorStreamCaptureInvalidated = 901,
  hipErrorStreamCaptureMerge = 902,
  hipErrorStreamCaptureUnmatched = 903,
  hipErrorStreamCaptureUnjoined = 904,
  hipErrorStreamCaptureIsolation = 905,
  hipErrorIllegalState = 906,
};
typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
typedef struct ihipGraph *hipGraph_t;
typedef struct hipGraphExec *hipGraphExec_t;
typedef struct hipGraphNode *hipGraphNode_t;
typedef enum { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed } hipStreamCaptureMode;
typedef enum { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault } hipMemcpyKind;
#define hipStreamNonBlocking 0x01
#define hipEventDisableTiming 0x02

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *err_node, char *log, size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t x);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipDeviceSynchronize(void);
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind);
const char *hipGetErrorString(hipError_t e);

// What the column library's host unit (csrc/ms_api.hip) needs besides the executor's calls:
// its one device-side array becomes a host array.
#define __device__
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (reinterpret_cast<const void *>(&(x)))
struct hipDeviceProp_t {
  int multiProcessorCount;
};
hipError_t hipGetDevice(int *device);
hipError_t hipGetDeviceProperties(hipDeviceProp_t *prop, int device);
hipError_t hipGetSymbolAddress(void **ptr, const void *symbol);
hipError_t hipMallocAsync(void **ptr, size_t bytes, hipStream_t s);
hipError_t hipFreeAsync(void *ptr, hipStream_t s);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipGetLastError(void);
