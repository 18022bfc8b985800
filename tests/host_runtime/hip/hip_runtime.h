// Stand-in HIP header for the host-side runtime test: lets the library's host
// code (plans, submission, tickets, check bookkeeping, batch tables) build with
// g++ and run under AddressSanitizer / UBSan on a machine without a GPU.
// "Device" memory is host memory, copies are memcpy, kernels are the stubs of
// launch_stubs.cpp.  Like HIP, querying an event that has not finished returns
// hipErrorNotReady and records it as the thread's last error.
#pragma once
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <cstddef>
#define __device__
#define __global__
#define __forceinline__ inline
#define __host__
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (&(x))
struct float2 { float x, y; };
struct double2 { double x, y; };
struct uint2 { unsigned x, y; };
struct uint4 { unsigned x, y, z, w; };
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorNotReady = 600, hipErrorInvalidValue = 1, hipErrorInvalidConfiguration = 9 };
typedef struct ihipStream_t *hipStream_t;
struct FakeEvent { int recorded; int polls; };
inline thread_local hipError_t g_fake_last = 0;
inline hipError_t hipGetLastError() { hipError_t e = g_fake_last; g_fake_last = 0; return e; }
typedef FakeEvent *hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum { hipHostMallocDefault = 0, hipEventDisableTiming = 2 };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1 };
inline const char *hipGetErrorString(hipError_t) { return "fake"; }
inline hipError_t hipHostMalloc(void **p, size_t n, unsigned) { *p = malloc(n); return hipSuccess; }
inline hipError_t hipMalloc(void **p, size_t n) { *p = malloc(n); return hipSuccess; }
inline hipError_t hipFree(void *p) { free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) { memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = new FakeEvent{0, 0}; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->recorded = 1; e->polls = 0; return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t e) { if (e->polls++ < 2) { g_fake_last = hipErrorNotReady; return hipErrorNotReady; } return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) { *p = const_cast<void *>(sym); return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int) { *v = 256; return hipSuccess; }
template <class T> T atomicAdd(T *p, T v) { T o = *p; *p += v; return o; }
