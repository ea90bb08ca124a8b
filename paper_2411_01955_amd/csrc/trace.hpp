// Kernel tracing hooks (see trace.hip).
#pragma once

#include <string>

#include "common.hpp"

namespace pnp {

bool trace_on();
void trace_enable(bool on);
std::string trace_read_json();

// Brackets one kernel launch with events on `s` while tracing is enabled.
class TraceScope {
 public:
  TraceScope(hipStream_t s, const char* name);
  ~TraceScope();
  TraceScope(const TraceScope&) = delete;
  TraceScope& operator=(const TraceScope&) = delete;

 private:
  hipStream_t stream_;
  const char* name_;
  bool active_;
  hipEvent_t a_{}, b_{};
};

}  // namespace pnp

// Launch a kernel on stream `s`, traced under the kernel's own name.
#define PNP_LAUNCH(kernel, grid, block, lds, s, ...)                        \
  do {                                                                     \
    ::pnp::TraceScope trace_scope_(s, #kernel);                            \
    hipLaunchKernelGGL(kernel, grid, block, lds, s, __VA_ARGS__);          \
    PNP_CHECK_LAUNCH();                                                    \
  } while (0)
