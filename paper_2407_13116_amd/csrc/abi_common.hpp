// Shared host-side helpers of the C ABI: the per-thread last-error string,
// argument checks and launch-error translation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <string>

namespace ksvd2 {

enum Status : int {
  KSVD2_OK = 0,
  KSVD2_EINVAL = -1,
  KSVD2_EDTYPE = -2,
  KSVD2_EHIP = -3,
  KSVD2_EWORKSPACE = -4,
};

std::string &last_error_ref();

inline int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error_ref() = buf;
  return code;
}

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// required pointer: non-null and aligned to its element size
#define KSVD2_REQ(ptr, align)                                                            \
  do {                                                                                   \
    if ((ptr) == nullptr) return ::ksvd2::fail(::ksvd2::KSVD2_EINVAL, "%s is null", #ptr); \
    if (!::ksvd2::aligned((ptr), (align)))                                               \
      return ::ksvd2::fail(::ksvd2::KSVD2_EINVAL, "%s is not %zu-byte aligned", #ptr,    \
                           (size_t)(align));                                             \
  } while (0)

// optional pointer: aligned when present
#define KSVD2_OPT(ptr, align)                                                         \
  do {                                                                                \
    if ((ptr) != nullptr && !::ksvd2::aligned((ptr), (align)))                        \
      return ::ksvd2::fail(::ksvd2::KSVD2_EINVAL, "%s is not %zu-byte aligned", #ptr, \
                           (size_t)(align));                                          \
  } while (0)

inline int launch_status(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(KSVD2_EHIP, "%s: %s", what, hipGetErrorString(e));
  return KSVD2_OK;
}

constexpr int kBlock = 256;  // threads per workgroup of the batched 2x2 kernels

inline unsigned grid_for(int64_t n, int block = kBlock) {
  return (unsigned)((n + block - 1) / block);
}

}  // namespace ksvd2
