// Device memory accounting of the library: every device allocation goes
// through dev_malloc / dev_free, which keep the bytes held by the process and
// refuse an allocation that would take that total past the cap read from
// the environment variable SOAP_MAX_DEVICE_BYTES (a byte count; unset, empty
// or 0 means no cap).  A refused allocation returns hipErrorOutOfMemory, so
// every caller reports it as SOAP_ERR_OOM, with dev_cap_note() saying why.
// The cap is read at each allocation, so a process can change it between
// calls.  The fixed array of the allocation-free entry point is not counted:
// it is part of the loaded code object, not an allocation.
#include <hip/hip_runtime.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <unordered_map>

#include "soap_internal.hpp"

namespace soap {

namespace {

std::mutex g_mu;
std::unordered_map<void*, size_t> g_sizes;
uint64_t g_held = 0;
thread_local std::string g_note;

// 0 = no cap; an unparsable value caps at 0 bytes (every allocation fails,
// with the note naming the value) rather than being ignored
bool read_cap(uint64_t* cap) {
  const char* s = std::getenv("SOAP_MAX_DEVICE_BYTES");
  *cap = 0;
  if (!s || !*s) return true;
  errno = 0;
  char* end = nullptr;
  const unsigned long long v = std::strtoull(s, &end, 10);
  if (errno != 0 || end == s || *end != '\0') return false;
  *cap = v;
  return true;
}

}  // namespace

hipError_t dev_malloc(void** p, size_t bytes) {
  *p = nullptr;
  uint64_t cap = 0;
  const bool ok = read_cap(&cap);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!ok || (cap != 0 && g_held + bytes > cap)) {
    char buf[256];
    if (!ok)
      std::snprintf(buf, sizeof buf, " (SOAP_MAX_DEVICE_BYTES is not a byte count)");
    else
      std::snprintf(buf, sizeof buf, " (%zu bytes more would pass SOAP_MAX_DEVICE_BYTES = %llu; %llu held)",
                    bytes, (unsigned long long)cap, (unsigned long long)g_held);
    g_note = buf;
    return hipErrorOutOfMemory;
  }
  g_note.clear();
  const hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess && *p) {
    g_sizes[*p] = bytes;
    g_held += bytes;
  }
  return e;
}

hipError_t dev_free(void* p) {
  if (!p) return hipSuccess;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_sizes.find(p);
    if (it != g_sizes.end()) {
      g_held -= it->second;
      g_sizes.erase(it);
    }
  }
  return hipFree(p);
}

uint64_t dev_bytes_held() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_held;
}

const char* dev_cap_note() { return g_note.c_str(); }

}  // namespace soap
