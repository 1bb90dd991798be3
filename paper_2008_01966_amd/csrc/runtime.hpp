// Library-internal services shared by the plan code (capi.cpp) and the request server
// (server.cpp).
#pragma once

#include <cstddef>

namespace cav {

// Device blocks from the process-wide cache of the library (hipMalloc only on a miss).
// release: the caller guarantees that no queued work still uses the block.
int device_block_acquire(size_t bytes, void** out);
void device_block_release(void* ptr, size_t bytes);

// Record the status and message of the calling thread's last error (cavity_last_error).
int record_error(int status, const char* msg);

}  // namespace cav
