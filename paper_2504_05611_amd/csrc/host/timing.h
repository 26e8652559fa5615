// Optional per-kernel timing: every library kernel launch can be bracketed by
// HIP events on its own stream; totals are read back on request.
#pragma once

#include <hip/hip_runtime.h>

namespace tmcs {

bool timing_on();
void timing_begin(const char* name, hipStream_t s, void** token);
void timing_end(void* token, hipStream_t s);

struct TimedLaunch {
  void* token = nullptr;
  hipStream_t s;
  TimedLaunch(const char* name, hipStream_t st) : s(st) {
    if (timing_on()) timing_begin(name, s, &token);
  }
  ~TimedLaunch() {
    if (token) timing_end(token, s);
  }
};

}  // namespace tmcs

// Launch a kernel, timing it when timing is enabled.
#define TMCS_LAUNCH(name, kernel, grid, block, lds, stream, ...)            \
  do {                                                                      \
    ::tmcs::TimedLaunch _tl(name, stream);                                  \
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);      \
  } while (0)
