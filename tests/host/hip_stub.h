// Interface of the host-only HIP stand-in (tests/host/hip_stub.cpp) for the sanitizer driver.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace stub {
struct Launch {
  const void* fn;
  unsigned gx, gy, gz, bx, by, bz;
  size_t shm;
  uintptr_t stream;
};
void* device_alloc(size_t bytes);        // a "device" allocation the buffer checks accept
std::vector<Launch> launches();          // kernel launches recorded so far
void clear_launches();
}  // namespace stub
