// Hooks of the host-only HIP model (test infrastructure).
#pragma once
#include <hip/hip_runtime.h>

#include <functional>

namespace model {
// Queue device work on stream s (a graph node while s is capturing).
void submit(hipStream_t s, std::function<void()> work);
bool capturing(hipStream_t s);
void synchronize();
}  // namespace model
