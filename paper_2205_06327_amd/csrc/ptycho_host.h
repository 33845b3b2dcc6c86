// ptycho_host.h -- host-side helpers shared by the translation units of the C
// ABI: the thread-local error message and the checks of caller buffers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ptycho {
namespace host {

// Records a printf-style message as the thread's last error and returns `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// PTYCHO_E_HIP with the runtime's message for `e`.
int hip_fail(hipError_t e, const char* what);
// The calling thread's last error message.
const char* last_error();
// PTYCHO_OK when [p, p + bytes) is device-accessible memory of `device` (or managed or pinned host
// memory) lying inside its allocation where the runtime knows it; a null p or bytes == 0 passes.
int check_buffer(int device, const void* p, size_t bytes, const char* what);
// Elements spanned by a [S][h][w] view with strides (slice_stride, ld), 0 when empty, saturating
// far beyond any allocation so that absurd strides fail check_buffer instead of wrapping around.
size_t span_elems(int64_t S, int64_t h, int64_t w, int64_t slice_stride, int64_t ld);

}  // namespace host
}  // namespace ptycho

#define PT_HIP(call)                                                \
  do {                                                              \
    hipError_t e_ = (call);                                         \
    if (e_ != hipSuccess) return ::ptycho::host::hip_fail(e_, #call); \
  } while (0)

#define PT_BUF(dev, p, bytes, what)                                          \
  do {                                                                       \
    int rc_ = ::ptycho::host::check_buffer((dev), (p), (bytes), (what));     \
    if (rc_ != PTYCHO_OK) return rc_;                                        \
  } while (0)
