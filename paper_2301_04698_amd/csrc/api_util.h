// Error reporting shared by the C ABI translation units: a thread-local
// message returned by les_last_error() and the HIP status checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <exception>
#include <new>
#include <string>

#include "les.h"

namespace lesmi {

inline thread_local std::string g_error;

inline int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

// Runs an entry point's body so that no C++ exception leaves the C ABI:
// host allocation failure and any other exception become LES_ERR_STATE.
template <typename F>
int guarded(F &&body) {
  try {
    return body();
  } catch (const std::bad_alloc &) {
    return fail(LES_ERR_STATE, "out of host memory");
  } catch (const std::exception &e) {
    return fail(LES_ERR_STATE, "internal error: %s", e.what());
  } catch (...) {
    return fail(LES_ERR_STATE, "internal error");
  }
}

}  // namespace lesmi

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return lesmi::fail(LES_ERR_HIP, "%s failed: %s (%s:%d)", #expr,                    \
                         hipGetErrorString(e_), __FILE__, __LINE__);                     \
  } while (0)

#define LAUNCH_TRY()                                                                     \
  do {                                                                                   \
    hipError_t e_ = hipGetLastError();                                                   \
    if (e_ != hipSuccess)                                                                \
      return lesmi::fail(LES_ERR_HIP, "kernel launch failed: %s (%s:%d)",               \
                         hipGetErrorString(e_), __FILE__, __LINE__);                     \
  } while (0)
