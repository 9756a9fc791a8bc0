// Internal declarations of libsoap: context layout, kernel launchers and the
// device helpers shared by the kernels.  Nothing here is part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "soap.h"

namespace soap {

constexpr double C_KMS = 299792.458;
// second radiation constant h c / k_B, m K (exact in SI 2019)
constexpr double C2_MK = 1.438776877e-2;
constexpr double DEG = 3.14159265358979323846 / 180.0;

constexpr int MAX_REGIONS = 64;
constexpr int MAX_MU = 64;
constexpr int MAX_GRID = 4096;
constexpr int MAX_PHASES = 1 << 20;

// apply kernel shape: R pixels per thread, PC phases per chunk, JW offsets
// per virtual group window, 256 threads per block.
constexpr int APPLY_R = 4;
constexpr int APPLY_PC = 8;
constexpr int APPLY_JW = 8;
constexpr int APPLY_THREADS = 256;
constexpr int APPLY_TILE = APPLY_R * APPLY_THREADS;

// region record as the kernels read it (device copy of soap_region)
struct Region {
  int type;
  int pad;
  double lat_deg, lon_deg, radius, contrast;
};

// one virtual group of a phase chunk: source group g = type*B + bin (type 0 =
// quiet removal), window of APPLY_JW offsets starting at jlo, and for each
// phase of the chunk the range [off[p], off[p+1]) of its entries
struct VGroup {
  int g;
  int jlo;
  int off[APPLY_PC + 1];
};

// one run of <= 4 consecutive taps inside a window: code = q0*4 + (w-1)
template <typename T>
struct Entry {
  int code;
  int pad;
  T k[4];
};

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace soap

struct soap_ctx {
  int device = 0;
  bool hip_used = false;
  hipStream_t stream = nullptr;
  std::string err;

  // star
  int N = 0, B = 0;
  int64_t P = 0;
  double vsini = 0, incl = 0, u1 = 0, u2 = 0, ln0 = 0, dln = 0;
  int prec = SOAP_PREC_FP64, cmode = SOAP_CONTRAST_SCALAR;
  double teff = 0, dt_spot = 0, dt_fac[3] = {0, 0, 0};
  std::vector<double> mu_bins;
  bool has_type[3] = {false, false, false};
  int jmin = 0, jmax = 0, J = 0;  // tap offset range [jmin, jmax], J = jmax - jmin + 1
  size_t esize = 8;               // element size of spectra / flux

  // resident device state
  void* d_spec[3] = {nullptr, nullptr, nullptr};  // [B][P]
  double* d_mu = nullptr;                          // [B]
  int* d_col_c = nullptr;                          // [N]
  double* d_col_w = nullptr;                       // [N]
  double* d_colW = nullptr;                        // [N][B] quiet column weights
  double* d_Kq = nullptr;                          // [B][J] quiet taps
  double* d_Q = nullptr;                           // [P]
  void* d_con_spot = nullptr;                      // [P] (PLANCK)
  void* d_con_fac = nullptr;                       // [B][P] (PLANCK)

  // per-call workspace (grown on demand, freed by soap_destroy)
  soap::Workspace ws_K;        // [n_phases][G][J] double
  soap::Workspace ws_vg;       // [n_chunks][G*ceil(J/JW)] VGroup
  soap::Workspace ws_nvg;      // [n_chunks] int
  soap::Workspace ws_ent;      // [n_chunks][max entries] Entry<T>
  soap::Workspace ws_flux;     // host-output staging for fluxes
  soap::Workspace ws_ccf;      // partial CCFs
  soap::Workspace ws_ccfout;   // [n_spec][n_v] double
  soap::Workspace ws_rv;       // [n_spec] soap_rv
  soap::Workspace ws_mask;     // [n_lines] double2 (u, w)
  soap::Workspace ws_specin;   // host-input staging for ccf
  void* pinned = nullptr;      // host staging for the mask upload
  size_t pinned_bytes = 0;
  hipEvent_t pinned_done = nullptr;
  // ring of pinned parameter slots (regions + phases) read in place by the
  // weights kernel; a slot is rewritten only after the kernel that read it
  // has finished
  static constexpr int NSLOT = 4;
  void* slot[NSLOT] = {nullptr, nullptr, nullptr, nullptr};
  size_t slot_bytes[NSLOT] = {0, 0, 0, 0};
  hipEvent_t slot_done[NSLOT] = {nullptr, nullptr, nullptr, nullptr};
  int slot_next = 0;

  // profiling (soap_profile_enable / soap_profile_read)
  bool prof = false;
  struct Pending {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  double stage_ms[5] = {0, 0, 0, 0, 0};
  int64_t active_calls = 0, ccf_calls = 0;
  int last_phases = 0, last_effect = 0, last_vg_cap = 0;

  // cached mask
  std::vector<double> mask_lnl, mask_w;
  double mask_h = 0, mask_v0 = 0, mask_dv = 0;
  int mask_nv = 0;
  bool mask_valid = false;
};

namespace soap {

// ---- launchers (each enqueues on ctx->stream; return hipError_t) ----------
hipError_t launch_geom(soap_ctx* c);
hipError_t launch_contrast(soap_ctx* c);
hipError_t launch_quiet(soap_ctx* c);
hipError_t launch_weights(soap_ctx* c, const Region* d_reg, int n_reg, const double* d_ph, int n_ph,
                          int effect, double* d_K);
hipError_t launch_compact(soap_ctx* c, const double* d_K, int n_ph, VGroup* d_vg, int* d_nvg,
                          void* d_ent, int vg_cap, int ent_cap);
hipError_t launch_apply(soap_ctx* c, const VGroup* d_vg, const int* d_nvg, const void* d_ent,
                        int vg_cap, int ent_cap, int n_ph, int effect, void* d_flux);
hipError_t launch_q_convert(soap_ctx* c, void* out);
hipError_t launch_ccf(soap_ctx* c, const void* d_flux, int64_t n_spec, const double* d_mask,
                      int n_lines, double* d_part, double* d_ccf);
hipError_t launch_gfit(soap_ctx* c, const double* d_ccf, int64_t n_spec, soap_rv* d_rv);
hipError_t launch_mask_prep(soap_ctx* c, const double* d_lnl, const double* d_w, int n, double* d_mask);

int ccf_line_blocks(int n_lines);

// ---- device helpers ---------------------------------------------------------
#ifdef __HIP_DEVICE_COMPILE__
#define SOAP_DEV __device__ __forceinline__
#else
#define SOAP_DEV __host__ __device__ inline
#endif

// Decision arithmetic (which cells are on the disk, which bin, which region)
// is done in double with every product and sum rounded separately, so that a
// reader evaluating the same expressions in IEEE double gets the same
// decisions.
SOAP_DEV double cell_coord(int i, int n) {
#pragma clang fp contract(off)
  return (2.0 * i + 1.0) / n - 1.0;
}

SOAP_DEV double limb_dark(double mu, double u1, double u2) {
#pragma clang fp contract(off)
  double om = 1.0 - mu;
  return 1.0 - u1 * om - u2 * om * om;
}

SOAP_DEV int nearest_bin(double mu, const double* mu_b, int B) {
#pragma clang fp contract(off)
  int bi = 0;
  double best = fabs(mu - mu_b[0]);
  for (int b = 1; b < B; ++b) {
    double d = fabs(mu - mu_b[b]);
    if (d < best) {
      best = d;
      bi = b;
    }
  }
  return bi;
}

// observer-frame unit vector of a region centre at a rotation phase
SOAP_DEV void region_centre(double lat, double lon, double phase, double incl, double* cx, double* cy,
                            double* cz) {
#pragma clang fp contract(off)
  double th = lat * DEG;
  double psi = (lon + 360.0 * phase) * DEG;
  double inc = incl * DEG;
  double X = cos(th) * sin(psi);
  double Y = sin(th);
  double Z = cos(th) * cos(psi);
  *cx = X;
  *cy = Y * sin(inc) - Z * cos(inc);
  *cz = Y * cos(inc) + Z * sin(inc);
}

}  // namespace soap
