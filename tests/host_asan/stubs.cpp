// CPU stand-ins for the HIP runtime calls of libqtn's host code, so that the
// planner, the workspace layout, the launch logic, the autotuner and the
// C ABI can run under AddressSanitizer on a machine without a GPU.  Memory
// calls map to host memory; kernel launches, events and synchronisation do
// nothing (no device results are produced or checked here).
#include <hip/hip_runtime_api.h>

#include <cstdlib>
#include <cstring>

extern "C" {
static void *fat_handle[4];
void **__hipRegisterFatBinary(const void *) { return fat_handle; }
void __hipUnregisterFatBinary(void **) {}
void __hipRegisterFunction(void **, const void *, char *, const char *, unsigned int, void *, void *, void *,
                           void *, int *) {}
void __hipRegisterVar(void **, void *, char *, const char *, int, size_t, int, int) {}
hipError_t __hipPushCallConfiguration(dim3, dim3, size_t, hipStream_t) { return hipSuccess; }
hipError_t __hipPopCallConfiguration(dim3 *, dim3 *, size_t *, hipStream_t *) { return hipSuccess; }
hipError_t hipLaunchKernel(const void *, dim3, dim3, void **, size_t, hipStream_t) { return hipSuccess; }
hipError_t hipMalloc(void **p, size_t n) {
  *p = aligned_alloc(256, (n + 255) & ~size_t(255));
  memset(*p, 0, n);
  return hipSuccess;
}
hipError_t hipFree(void *p) {
  free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
  memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) {
  memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemset(void *d, int v, size_t n) {
  memset(d, v, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) {
  memset(d, v, n);
  return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) {
  *p = malloc(n);
  memset(*p, 0, n);
  return hipSuccess;
}
hipError_t hipHostGetDevicePointer(void **d, void *h, unsigned int) {
  *d = h;
  return hipSuccess;
}
hipError_t hipHostFree(void *p) {
  free(p);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
  *e = (hipEvent_t)malloc(8);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
  *e = (hipEvent_t)malloc(8);
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  free((void *)e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
  *ms = 0.01f;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  *s = (hipStream_t)malloc(8);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  free((void *)s);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamQuery(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
  *g = (hipGraph_t)malloc(8);
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *ge, hipGraph_t, hipGraphNode_t *, char *, size_t) {
  *ge = (hipGraphExec_t)malloc(8);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) {
  free((void *)g);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t g) {
  free((void *)g);
  return hipSuccess;
}
hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "host stand-in"; }
hipError_t hipFuncSetAttribute(const void *, hipFuncAttribute, int) { return hipSuccess; }
// the no-allocation entry point's file-scope array: one host block
static char *symbuf;
hipError_t hipGetSymbolAddress(void **p, const void *) {
  if (!symbuf) symbuf = (char *)aligned_alloc(256, size_t(64) << 20);
  *p = symbuf;
  return hipSuccess;
}
}
