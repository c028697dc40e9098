// A host-only stand-in for the HIP runtime, for the sanitizer build of libwolf's host code (test
// infrastructure). "Device" allocations are host memory from a table, so the buffer checks of the
// C ABI see real allocations; kernel launches are recorded (grid, block, LDS) and not executed;
// streams, events and graphs are plain handles. Nothing here is compiled into the library.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <vector>

#include "hip_stub.h"

namespace {
struct Alloc {
  char* p;
  size_t n;
};
// Held through pointers that are never freed, so that the allocations stay reachable from a global
// until the process ends (no static destructor runs before the leak check).
// The library's module constructors register device variables before this file's globals would be
// initialised, so every table is built on first use.
std::mutex g_mu;
std::vector<Alloc>& allocs() {
  static std::vector<Alloc>& v = *new std::vector<Alloc>;
  return v;
}
std::vector<stub::Launch>& launches_log() {
  static std::vector<stub::Launch>& v = *new std::vector<stub::Launch>;
  return v;
}
std::set<uintptr_t>& capturing() {  // streams between BeginCapture and EndCapture
  static std::set<uintptr_t>& v = *new std::set<uintptr_t>;
  return v;
}
thread_local std::vector<stub::Launch> t_config;
int g_handles = 0;

std::vector<std::pair<const void*, void*>>& g_vars() {
  static std::vector<std::pair<const void*, void*>>& v = *new std::vector<std::pair<const void*, void*>>;
  return v;
}

const Alloc* find(const void* q) {
  for (const auto& a : allocs())
    if ((const char*)q >= a.p && (const char*)q < a.p + a.n) return &a;
  return nullptr;
}
void* handle() { return reinterpret_cast<void*>((uintptr_t)(0x1000 + 16 * ++g_handles)); }
}  // namespace

namespace stub {
void* device_alloc(size_t bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  char* p = static_cast<char*>(std::calloc(bytes ? bytes : 1, 1));
  allocs().push_back(Alloc{p, bytes});
  return p;
}
std::vector<Launch> launches() {
  std::lock_guard<std::mutex> lk(g_mu);
  return launches_log();
}
void clear_launches() {
  std::lock_guard<std::mutex> lk(g_mu);
  launches_log().clear();
}
}  // namespace stub

extern "C" {

hipError_t hipMalloc(void** p, size_t n) {
  if (!p) return hipErrorInvalidValue;
  *p = stub::device_alloc(n);
  return hipSuccess;
}

hipError_t hipPointerGetAttributes(hipPointerAttribute_t* attr, const void* q) {
  std::lock_guard<std::mutex> lk(g_mu);
  const Alloc* a = find(q);
  if (!a) return hipErrorInvalidValue;
  std::memset(attr, 0, sizeof *attr);
  attr->type = hipMemoryTypeDevice;
  attr->device = 0;
  attr->devicePointer = const_cast<void*>(q);
  return hipSuccess;
}

hipError_t hipMemGetAddressRange(hipDeviceptr_t* base, size_t* size, hipDeviceptr_t q) {
  std::lock_guard<std::mutex> lk(g_mu);
  const Alloc* a = find(q);
  if (!a) return hipErrorInvalidValue;
  *base = a->p;
  *size = a->n;
  return hipSuccess;
}

hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "stub error"; }

hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
  std::memcpy(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const Alloc* a = find(dst);
    if (!a || (const char*)dst + n > a->p + a->n) {
      std::fprintf(stderr, "stub: hipMemsetAsync outside an allocation\n");
      std::abort();
    }
  }
  std::memset(dst, v, n);
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
  *e = static_cast<hipEvent_t>(handle());
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 1.0f;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = static_cast<hipStream_t>(handle());
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  std::lock_guard<std::mutex> lk(g_mu);
  capturing().insert((uintptr_t)s);
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  std::lock_guard<std::mutex> lk(g_mu);
  capturing().erase((uintptr_t)s);
  *g = static_cast<hipGraph_t>(handle());
  return hipSuccess;
}
hipError_t hipStreamIsCapturing(hipStream_t s, hipStreamCaptureStatus* st) {
  std::lock_guard<std::mutex> lk(g_mu);
  *st = capturing().count((uintptr_t)s) ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  *x = static_cast<hipGraphExec_t>(handle());
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }

// Kernel launches: the <<<>>> stubs push the configuration, then call hipLaunchKernel.
hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shm, hipStream_t s) {
  t_config.push_back(stub::Launch{nullptr, grid.x, grid.y, grid.z, block.x, block.y, block.z, shm, (uintptr_t)s});
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* grid, dim3* block, size_t* shm, hipStream_t* s) {
  if (t_config.empty()) return hipErrorInvalidValue;
  const stub::Launch c = t_config.back();
  t_config.pop_back();
  *grid = dim3(c.gx, c.gy, c.gz);
  *block = dim3(c.bx, c.by, c.bz);
  *shm = c.shm;
  *s = reinterpret_cast<hipStream_t>(c.stream);
  return hipSuccess;
}
hipError_t hipLaunchKernel(const void* f, dim3 grid, dim3 block, void**, size_t shm, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  launches_log().push_back(stub::Launch{f, grid.x, grid.y, grid.z, block.x, block.y, block.z, shm, (uintptr_t)s});
  return hipSuccess;
}
void** __hipRegisterFatBinary(const void*) {
  static void* module = nullptr;
  return &module;
}
void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int, uint3*, uint3*, dim3*, dim3*, int*) {}
void __hipUnregisterFatBinary(void**) {}

// Device variables: the host stand-in of each registered variable maps to a "device" allocation of
// its size, which hipGetSymbolAddress returns (as the runtime returns the device copy's address).
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
  std::lock_guard<std::mutex> lk(g_mu);
  char* p = static_cast<char*>(std::calloc(size ? size : 1, 1));
  allocs().push_back(Alloc{p, size});
  g_vars().push_back(std::make_pair(static_cast<const void*>(var), static_cast<void*>(p)));
}
hipError_t hipGetSymbolAddress(void** dev, const void* symbol) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& v : g_vars())
    if (v.first == symbol) {
      *dev = v.second;
      return hipSuccess;
    }
  return hipErrorInvalidSymbol;
}

}  // extern "C"
