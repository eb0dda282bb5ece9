// Stand-in for the HIP runtime in the host-only test build of libgw's C ABI
// layer (tests/test_host_build.py).  "Device" memory is host memory
// (zero-filled), copies are memcpy, streams, events and graphs are handles
// that do nothing, and no kernel exists: the kernel launchers are stubs that
// return success.  It lets the argument checks, status codes, sticky errors,
// forced faults and the serving state machine run on a machine without a GPU,
// under the address and undefined-behaviour sanitizers.  Never part of the
// library.
#pragma once

#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNoDevice = 100,
    hipErrorInvalidDevice = 101,
    hipErrorLaunchFailure = 719,
    hipErrorUnknown = 999
} hipError_t;

typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
typedef struct ihipGraph *hipGraph_t;
typedef struct hipGraphExec *hipGraphExec_t;
typedef struct hipGraphNode *hipGraphNode_t;
typedef struct ihipMemPoolHandle_t *hipMemPool_t;
typedef enum { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice } hipMemcpyKind;
typedef enum { hipStreamCaptureStatusNone, hipStreamCaptureStatusActive } hipStreamCaptureStatus;
typedef enum { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed } hipStreamCaptureMode;
typedef enum { hipMemPoolAttrReleaseThreshold = 4 } hipMemPoolAttr;

#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u

namespace hipstub {
// one live handle object per kind; the library only compares and passes them
inline void *handle() {
    static char h[64];
    return h;
}
}  // namespace hipstub

inline const char *hipGetErrorString(hipError_t e) {
    switch (e) {
        case hipSuccess: return "no error";
        case hipErrorOutOfMemory: return "out of memory";
        case hipErrorLaunchFailure: return "unspecified launch failure";
        case hipErrorInvalidValue: return "invalid argument";
        default: return "unknown error";
    }
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
inline hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
inline hipError_t hipGetDeviceCount(int *n) {
    *n = 1;
    return hipSuccess;
}
typedef enum { hipDeviceAttributeMultiprocessorCount = 63 } hipDeviceAttribute_t;
inline hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int d) {
    *v = 256;
    return d == 0 ? hipSuccess : hipErrorInvalidDevice;
}
inline hipError_t hipMemGetInfo(size_t *fr, size_t *tot) {
    *fr = (size_t)64 << 30;
    *tot = (size_t)64 << 30;
    return hipSuccess;
}
inline hipError_t hipMalloc(void **p, size_t b) {
    *p = calloc(1, b ? b : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void *p) {
    free(p);
    return hipSuccess;
}
inline hipError_t hipMallocAsync(void **p, size_t b, hipStream_t) { return hipMalloc(p, b); }
inline hipError_t hipFreeAsync(void *p, hipStream_t) { return hipFree(p); }
inline hipError_t hipMemcpy(void *d, const void *s, size_t b, hipMemcpyKind) {
    if (b) memmove(d, s, b);
    return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t b, hipMemcpyKind k, hipStream_t) {
    return hipMemcpy(d, s, b, k);
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = (hipStream_t)hipstub::handle();
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) {
    *e = (hipEvent_t)hipstub::handle();
    return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
    *ms = 1.0f;
    return hipSuccess;
}
inline hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus *c) {
    *c = hipStreamCaptureStatusNone;
    return hipSuccess;
}
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
typedef enum { hipStreamAddCaptureDependencies = 0, hipStreamSetCaptureDependencies } hipStreamUpdateCaptureDependenciesFlags;
inline hipError_t hipStreamGetCaptureInfo_v2(hipStream_t, hipStreamCaptureStatus *c, unsigned long long *id,
                                             hipGraph_t *g, const hipGraphNode_t **d, size_t *n) {
    *c = hipStreamCaptureStatusNone;
    if (id) *id = 0;
    if (g) *g = nullptr;
    if (d) *d = nullptr;
    if (n) *n = 0;
    return hipSuccess;
}
inline hipError_t hipStreamUpdateCaptureDependencies(hipStream_t, hipGraphNode_t *, size_t, unsigned) { return hipSuccess; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
    *g = (hipGraph_t)hipstub::handle();
    return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t, void *, char *, size_t) {
    *x = (hipGraphExec_t)hipstub::handle();
    return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipGraphGetNodes(hipGraph_t, hipGraphNode_t *, size_t *n) {
    *n = 0;  // nothing is ever captured here
    return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
inline hipError_t hipDeviceGetDefaultMemPool(hipMemPool_t *p, int) {
    *p = (hipMemPool_t)hipstub::handle();
    return hipSuccess;
}
inline hipError_t hipMemPoolSetAttribute(hipMemPool_t, hipMemPoolAttr, void *) { return hipSuccess; }
inline hipError_t hipMemPoolTrimTo(hipMemPool_t, size_t) { return hipSuccess; }
