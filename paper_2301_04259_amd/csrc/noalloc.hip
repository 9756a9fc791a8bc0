// Allocation-free CCF and fit (soap_ccf_rv_noalloc in include/soap.h).
//
// soap_ccf_rv keeps the partial CCFs of its line blocks (and, without a
// caller CCF buffer, the summed CCF rows) in context workspace that it grows
// with hipMalloc.  This variant runs the same two kernels with that scratch
// in a file-scope device array instead, so it allocates nothing: for callers
// that cannot allocate (code under stream capture, serving loops, harnesses
// that forbid it).  The array's device address is looked up once per device
// at soap_grid_init, with that device current; host code only ever passes
// that address, never the array's name.  Every call on a device shares the
// device's array, so calls that overlap on one device race.
#include <mutex>

#include "soap_internal.hpp"

#define SOAP_API extern "C" __attribute__((visibility("default")))

namespace {

// 32 MiB: the FP32 partial CCFs of the headline mask (125 line blocks x 161
// velocities) for about 400 spectra
constexpr size_t SCRATCH_BYTES = size_t(32) << 20;
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

struct DeviceScratch {
  bool looked_up = false;
  hipError_t status = hipErrorNotInitialized;
  void* ptr = nullptr;  // device address of this device's copy of scratch
};

std::mutex g_mu;
DeviceScratch g_scratch[MAX_DEVICES];

}  // namespace

namespace soap {

hipError_t scratch_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceScratch& d = g_scratch[device];
  if (!d.looked_up) {
    void* p = nullptr;
    d.status = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    d.ptr = d.status == hipSuccess ? p : nullptr;
    d.looked_up = true;
  }
  return d.status;
}

}  // namespace soap

SOAP_API soap_status soap_ccf_rv_noalloc(soap_ctx* c, const void* flux, int64_t n_spec, const soap_mask* mask,
                                         double* ccf_out, soap_rv* rv_out) {
  if (!c) return SOAP_ERR_ARG;
  if (!flux || !mask) {
    c->err = "flux or mask is NULL";
    return SOAP_ERR_ARG;
  }
  if (n_spec < 1 || n_spec > (int64_t(1) << 24)) {
    c->err = "n_spec must be in [1, 2^24]";
    return SOAP_ERR_ARG;
  }
  if (!soap::mask_is_cached(c, mask)) {
    c->err = "soap_ccf_rv_noalloc needs the mask already set on the context: call soap_ccf_rv with it first";
    return SOAP_ERR_STATE;
  }
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const DeviceScratch& d = (c->device >= 0 && c->device < MAX_DEVICES) ? g_scratch[c->device] : DeviceScratch();
    if (!d.looked_up || d.status != hipSuccess) {
      c->err = std::string("no scratch on this device: hipGetSymbolAddress failed: ") +
               hipGetErrorString(d.looked_up ? d.status : hipErrorNotInitialized);
      return SOAP_ERR_HIP;
    }
    base = d.ptr;
  }
  const int nl = c->ccf_nl;  // the lines in the tables (those that reach the spectrum)
  const size_t rows = (size_t)n_spec * c->mask_nv;
  const size_t part_bytes = c->esize * rows * soap::ccf_line_blocks(nl);
  const size_t ccf_bytes = ccf_out ? 0 : sizeof(double) * rows;
  const size_t part_al = (part_bytes + 255) / 256 * 256;
  if (part_al + ccf_bytes > SCRATCH_BYTES) {
    char msg[256];
    std::snprintf(msg, sizeof msg,
                  "n_spec %lld needs %zu bytes of scratch for this mask, beyond the %zu available", (long long)n_spec,
                  part_al + ccf_bytes, SCRATCH_BYTES);
    c->err = msg;
    return SOAP_ERR_UNSUPPORTED;
  }
  void* part = base;
  double* ccf = ccf_out ? ccf_out : reinterpret_cast<double*>(static_cast<unsigned char*>(base) + part_al);
  hipError_t e = soap::launch_ccf(c, flux, n_spec, nl, part);
  if (e == hipSuccess) e = soap::launch_ccf_fit(c, nl, part, n_spec, ccf, rv_out);
  if (e != hipSuccess) {
    c->err = std::string("CCF launch failed: ") + hipGetErrorString(e);
    return SOAP_ERR_HIP;
  }
  return SOAP_OK;
}
