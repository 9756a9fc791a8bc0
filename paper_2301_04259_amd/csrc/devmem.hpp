// Device allocations of the library (devmem.cpp): they count the bytes the
// process holds and refuse, as hipErrorOutOfMemory, one that would pass the
// SOAP_MAX_DEVICE_BYTES cap; dev_cap_note() is the reason of the calling
// thread's last refusal ("" after an allocation that was not refused).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace soap {

hipError_t dev_malloc(void** p, size_t bytes);
hipError_t dev_free(void* p);
uint64_t dev_bytes_held();
const char* dev_cap_note();

}  // namespace soap
