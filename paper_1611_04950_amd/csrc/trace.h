// Kernel tracing: while enabled, each hot-path launch is bracketed by two HIP
// events recorded on its stream; durations are summed per kernel name when
// read.  Disabled, the cost is one relaxed atomic load per launch.
#pragma once

#include <hip/hip_runtime.h>

namespace slp {

bool trace_enabled();
void trace_mark_begin(const char *name, hipStream_t st);
void trace_mark_end(hipStream_t st);

}  // namespace slp

#define SLP_LAUNCH(name, kern, grid, block, shm, st, ...)          \
  do {                                                              \
    const bool tr_ = slp::trace_enabled();                          \
    if (tr_) slp::trace_mark_begin(name, st);                       \
    hipLaunchKernelGGL(kern, grid, block, shm, st, __VA_ARGS__);    \
    if (tr_) slp::trace_mark_end(st);                               \
  } while (0)
