// Helpers shared by the C ABI translation units: the thread-local error
// message, status returns, allocation with fault injection, device checks,
// handle teardown and scoped device buffers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../include/finger.h"
#include "internal.h"

namespace finger {
namespace abi {

using finger::Tables;

inline thread_local std::string g_err;

inline int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

inline int ok() {
  g_err.clear();
  return FINGER_OK;
}

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) return fail(FINGER_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

// Allocation with an injectable failure (FINGER_FAULT_INJECT=alloc makes
// every allocation fail, to test the error path).
inline int dev_alloc(void** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (bytes == 0) return FINGER_OK;
  const char* fi = std::getenv("FINGER_FAULT_INJECT");
  if (fi != nullptr && std::strcmp(fi, "alloc") == 0)
    return fail(FINGER_ENOMEM, "allocation of %zu bytes for %s failed (injected)", bytes, what);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(FINGER_ENOMEM, "allocation of %zu bytes for %s failed: %s", bytes, what,
                hipGetErrorString(e));
  }
  return FINGER_OK;
}

inline int check_device(int* dev_out) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return fail(FINGER_ENODEV, "no HIP device available");
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(FINGER_ENODEV, "device %d is %s; this library is built for gfx950", dev,
                prop.gcnArchName);
  if (dev_out) *dev_out = dev;
  return FINGER_OK;
}

inline int cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 256;
  return cus;
}

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

inline int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

inline void free_tables(Tables* t) {
  if (t == nullptr) return;
  void* dev_ptrs[] = {t->data_owned, t->P, t->cc, t->pc, t->alpha, t->rho, t->codes, t->scale,
                      t->piv_ids, t->qprep_B, t->qprep_Bnorm, t->piv_b16, t->piv_norm, t->samples, t->xy, t->gate_w,
                      t->gate_b, t->h_row0, t->h_upper};
  for (void* p : dev_ptrs)
    if (p) (void)hipFree(p);
  std::free(t->P64_host);
  std::free(t->eig_host);
  delete t;
}

struct Guard {  // frees a half-built handle on error paths
  Tables* t;
  ~Guard() { free_tables(t); }
};

template <typename T>
struct DevBuf {  // scoped temporary device buffer
  T* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
  }
  ~DevBuf() { reset(); }
};

}  // namespace abi
}  // namespace finger
