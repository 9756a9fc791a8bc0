// Internal declarations of libsoap: context layout, kernel launchers and the
// device helpers shared by the kernels.  Nothing here is part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "devmem.hpp"
#include "soap.h"

namespace soap {

constexpr double C_KMS = 299792.458;
// second radiation constant h c / k_B in m K, from the exact SI 2019 values
// h = 6.62607015e-34 J s, c = 299792458 m/s, k_B = 1.380649e-23 J/K
constexpr double C2_MK = 1.4387768775039337e-2;
constexpr double DEG = 3.14159265358979323846 / 180.0;

constexpr int MAX_REGIONS = 64;
constexpr int MAX_MU = 64;
constexpr int MAX_GRID = 4096;
constexpr int MAX_PHASES = 1 << 20;
constexpr int MAX_J = 64;  // tap offsets per table row

// Apply kernel shape: a block of APPLY_WAVES waves covers a tile of
// APPLY_WAVES x 64 x R consecutive pixels for one chunk of PC phases; each
// wave walks the chunk's windows of APPLY_JW offsets over its own 64 x R
// pixels with R x PC accumulators per lane (64 floats or 16 doubles), so
// R = 64 / PC in FP32 (PC = 8 or 16) and R = 16 / PC in FP64 (PC = 4 or 8).
// PC is a property of the context's tap tables, chosen per context (the
// first value of each pair is the default).  Quiet spectrum and rows are
// padded to whole tiles of APPLY_TILE_MAX pixels.
constexpr int APPLY_JW = 4;
constexpr int APPLY_WAVES = 4;
constexpr int APPLY_TILE_MAX = 2048;
constexpr int PC_MAX = 16;
constexpr int PC_F32 = 8, PC_F32_WIDE = 16;
constexpr int PC_F64 = 4, PC_F64_WIDE = 8;
inline bool pc_valid(bool fp32, int pc) {
  return fp32 ? (pc == PC_F32 || pc == PC_F32_WIDE) : (pc == PC_F64 || pc == PC_F64_WIDE);
}
// bytes of a window record (16-byte header, APPLY_JW x pc taps)
constexpr int win_bytes(int pc, int esize) { return 16 + APPLY_JW * pc * esize; }
constexpr int WIN_BYTES_MAX = 16 + APPLY_JW * PC_F32_WIDE * 4;
template <typename T, int PC>
struct ApplyShape {
  static_assert((sizeof(T) == 4 && (PC == PC_F32 || PC == PC_F32_WIDE)) ||
                    (sizeof(T) == 8 && (PC == PC_F64 || PC == PC_F64_WIDE)),
                "phases per chunk");
  static constexpr int R = (sizeof(T) == 4 ? 64 : 16) / PC;  // pixels per lane
  static constexpr int TILE = APPLY_WAVES * 64 * R;           // pixels per block
  static constexpr int WB = win_bytes(PC, (int)sizeof(T));    // window record bytes
  static_assert(TILE <= APPLY_TILE_MAX && WB <= WIN_BYTES_MAX && APPLY_JW * PC / 2 <= 32, "shape");
};

// Padded rows of the local spectra and contrast arrays: PAD_FRONT copies of
// the first sample before it and copies of the last sample after it, so that
// every window the apply kernel reads is in bounds and the end-value hold of
// the interpolation comes for free.
constexpr int PAD_FRONT = 128;

// widest line-spread function of the resolution lowering, in pixels each side
constexpr int LSF_KMAX = 32;

// With differential rotation each cell has its own shift, so the per-wave
// tables of the weight and quiet kernels hold [rows][offsets]; their size
// bounds n_mu x shift range (3 rows per bin in split tables).
constexpr int DR_TAB_MAX = 1536;

// Column slabs of the per-phase weight kernel (one wave per column).
constexpr int SLAB_COLS = 4;
constexpr int WEIGHT_WAVES = 4;
constexpr int FINISH_THREADS = 512;
// fixed-point unit of the per-phase tap accumulators
// (2^-59: sums up to |x| < 16, quantum 1.7e-18)
constexpr double FX_ONE = 576460752303423488.0;        // 2^59
constexpr double FX_INV = 1.0 / 576460752303423488.0;  // 2^-59
// largest disk weight x contrast the fixed-point sums accept
constexpr double FX_RANGE = 15.9;

// region record as the kernels read it (device view of soap_region)
struct Region {
  int type;
  int pad;
  double lat_deg, lon_deg, radius, contrast;
};

// A window record: APPLY_JW tap offsets [jlo, jlo + APPLY_JW) of one group
// in one phase chunk, stored as a 16-byte header followed by the dense taps
// taps[q][p] (q < APPLY_JW, p < the chunk's phase count; zeros where a phase
// has no tap).  Bit (q * PC / 2 + k) of gmask: phase 2k or 2k + 1 of the
// chunk has a non-zero tap at offset jlo + q.
// Group g: paired tables g = (type - 1) * B + bin; split tables
// g = type * B + bin with type 0 the quiet removal.
struct WinHead {
  int t;    // surface type of the group (0 = quiet removal)
  int b;    // mu bin of the group
  int jlo;
  unsigned int gmask;
};
// window records staged in LDS per pass of the apply kernel
constexpr int APPLY_LDS_WIN = 96;
// phase chunks the apply kernel orders by work (more run in their natural order)
constexpr int APPLY_RANKED = 64;

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Line-spread function of the resolution lowering: w[k + K] for |k| <= K
struct LsfPlan {
  int K = 0;
  double sigma = 0.0;
  double w[2 * LSF_KMAX + 1] = {};
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
  int64_t Pstride = 0;  // padded row length (elements); row data starts at PAD_FRONT
  int n_tiles = 0;  // tiles of APPLY_TILE_MAX pixels (padding)
  int tune_depth = 2;   // windows in flight per wave (2 or 3)
  int tune_order = 0;   // item order: 0 heaviest chunk first, 1 tile by tile
  double vsini = 0, incl = 0, u1 = 0, u2 = 0, ln0 = 0, dln = 0;
  double diff_rot = 0;  // omega(theta) = omega_0 (1 + diff_rot sin^2 theta)
  double sin_i = 0, cos_i = 1;
  int prec = SOAP_PREC_FP64, cmode = SOAP_CONTRAST_SCALAR;
  double teff = 0, dt_spot = 0, dt_fac[3] = {0, 0, 0};
  std::vector<double> mu_bins;
  bool has_type[3] = {false, false, false};
  int jmin = 0, jmax = 0, J = 0;  // tap offset range [jmin, jmax], J = jmax - jmin + 1
  size_t esize = 8;               // element size of spectra / flux
  int pc = soap::PC_F64;          // phases per apply chunk of the next call's tables

  // resident device state (row pointers point at pixel 0 of row 0)
  void* d_spec_base[3] = {nullptr, nullptr, nullptr};
  void* d_spec[3] = {nullptr, nullptr, nullptr};  // [B][Pstride]
  double* d_mu = nullptr;                          // [B]
  int* d_col_c = nullptr;                          // [N]
  double* d_col_w = nullptr;                       // [N]
  double* d_colW = nullptr;                        // [N][B] quiet column weights
  double* d_Kq = nullptr;                          // [B][J] quiet taps
  unsigned long long* d_Kq_fx = nullptr;           // [B][J] fixed-point quiet taps (differential rotation)
  double* d_Q = nullptr;                           // [n_tiles * TILE]
  void* d_con_base = nullptr;
  void* d_con_spot = nullptr;                      // [Pstride] (PLANCK) or [B][Pstride] (ARRAY)
  void* d_con_fac = nullptr;                       // [B][Pstride] (PLANCK, ARRAY)
  int con_rows = 0;                                // rows of d_con_base
  int64_t con_spot_stride = 0;                     // 0: one spot row for every bin (PLANCK)
  double disk_weight = 0.0;                        // sum over cells of (2/N)^2 |I(mu)|
  void* d_ones = nullptr;                          // [n_tiles * TILE] of 1 (no-contrast operand)

  // per-call workspace (grown on demand, freed by soap_destroy)
  // Per-call tables (region parameters, tap accumulators and taps, window
  // records), in two sets used by alternate calls.  Their kernels run on
  // the side stream, so the tables of the next call are built while the
  // context stream still runs the previous call's later stages.
  struct PrepSet {
    soap::Workspace par;     // regions, per-phase region centres and bounding boxes
    soap::Workspace Kfx;     // [n_phases][G][J] fixed-point tap accumulators (kept zero)
    soap::Workspace K;       // [n_phases][G][J] double
    soap::Workspace mask64;  // [n_phases][G] bitmask of nonzero offsets
    soap::Workspace vg;      // [n_chunks][vg_cap] window records (win_bytes(pc) each)
    soap::Workspace nvg;     // [n_chunks] int
    bool kfx_dirty = false;  // a call stopped between accumulation and clearing
    hipEvent_t prep_done = nullptr;   // side stream: this set's tables are built
    hipEvent_t apply_done = nullptr;  // context stream: the apply that read them is done
  };
  PrepSet prep[2];
  int prep_next = 0, last_prep = 0;
  hipStream_t side = nullptr;  // stream of the per-call table kernels
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
  double stage_ms[6] = {0, 0, 0, 0, 0, 0};
  int64_t active_calls = 0, ccf_calls = 0;
  // resolution lowering of the synthesised spectra (0: off)
  double lsf_resolution = 0.0;
  soap::LsfPlan lsf;
  soap::Workspace ws_lsf;  // synthesis output before the lowering
  soap::Workspace ws_sg;   // surrogate RVs: mean-prediction CCFs, sensitivities, flags
  int last_phases = 0, last_effect = 0, last_vg_cap = 0, last_paired = 0, last_pc = 0;

  // cached mask
  std::vector<double> mask_lnl, mask_w;
  double mask_h = 0, mask_v0 = 0, mask_dv = 0;
  double mask_hole_px = 0;  // widest hole of the velocity grid, in pixels
  int mask_nv = 0;
  // CCF tables of the cached mask in ws_mask (built by ccf_build_tables):
  // byte offsets of the sections, batch count, pixels per hole, stage span
  size_t ccf_off_edges = 0, ccf_off_batch = 0, ccf_off_bfirst = 0;
  int ccf_nbatch = 0, ccf_npx = 2, ccf_stg = 256;
  size_t mask_blob_bytes = 0;  // bytes of the mask's tables in ws_mask
  int ccf_nl = 0;              // mask lines in the tables (those that reach the spectrum)
  bool mask_valid = false;
};

namespace soap {

// Per-call plan shared by the weight, compaction and apply launches.
struct Plan {
  int n_ph = 0;
  int effect = 0;
  int paired = 0;   // 1: one tap table per active (type, bin); removal implied
  int G = 0;        // groups per table: 2B (paired) or 3B (split)
  int n_slabs = 0;
  int n_chunks = 0;
  int vg_cap = 0;   // virtual groups per chunk
  int pc = 0;       // phases per chunk of the tables
};

// ---- launchers (each enqueues on ctx->stream; return hipError_t) ----------
hipError_t launch_geom(soap_ctx* c);
hipError_t launch_pad(soap_ctx* c);
hipError_t launch_contrast(soap_ctx* c);
hipError_t launch_ones(soap_ctx* c);
hipError_t launch_quiet(soap_ctx* c);
// outputs and scratch of the weight kernel
struct WeightsOut {
  Region* reg;               // [n_regions] device copy of the regions
  int2* pj;                  // [n_phases] (first region, count) per phase, or unused
  double4* cen;              // [n_phases][max regions per phase] centres (x, y, z) and cos(alpha)
  int4* box;                 // [n_phases] disk-cell bounding box of the visible caps
  unsigned long long* Kfx;   // [n_phases][G][J] fixed-point taps, zero between calls
  double* K;                 // [n_phases][G][J] taps
  unsigned long long* mask;  // [n_phases][G] non-zero offsets
  unsigned char* wins;       // [n_chunks][vg_cap] window records
  int* nvg;                  // [n_chunks] windows per chunk
};
hipError_t launch_weights(soap_ctx* c, const Plan& pl, const Region* d_reg, int n_reg, int max_reg,
                          const double* d_ph, const int2* d_pj, const WeightsOut& o, hipStream_t st);
hipError_t launch_finish(soap_ctx* c, const Plan& pl, const WeightsOut& o, hipStream_t st);

// Arguments of the table kernels for one configuration (region parameters,
// weights, tap lists); the batched forms take an array of them.
struct ParamsArgs {
  int N, n_reg, max_reg, n_ph;
  double incl, diff_rot;
  const Region* reg;
  const double* phases;
  const int2* pj;
  Region* reg_out;
  int2* pj_out;
  double4* cen;
  int4* box;
};
struct WeightsArgs {
  int N, B, J, jmin, G, paired, n_slabs, effect, n_reg_all, max_reg;
  double u1, u2;
  const double* mu_b;
  const int* col_c;
  const double* col_w;
  const Region* reg;
  const int2* pj;
  const double4* cen;
  const int4* pbox;
  unsigned long long* Kfx;
};
struct FinishArgs {
  int n_ph, PC, G, J, jmin, B, paired, vg_cap;
  unsigned long long* Kfx;
  double* K;
  unsigned long long* mask;
  unsigned char* wins;
  int* nvg;
};

// Table kernels of many configurations as work-list launches: one launch per
// kernel (and per precision, and per finish mode), each block finding its
// configuration by a binary search over the configurations' block offsets.
// Configurations with differential rotation are not batched here (their
// weight kernel takes per-cell shifts); table_batch_add refuses them.
struct TableBatchCfg {
  soap_ctx* c;
  Plan pl;
  const Region* d_reg;
  int n_reg, max_reg;
  const double* d_ph;
  WeightsOut o;
  const Region* h_reg;  // host copies of the regions and phases: the weight
  const double* h_ph;   // launch lists only the slabs the caps can reach
};
struct TableBatch {
  // [kernel][variant]: params (1 variant), weights (FP32, FP64), finish
  // (FP32 / FP64 x tables in LDS or not)
  struct Launch {
    int n_cfg = 0, n_blocks = 0;
    size_t lds = 0;
    void* args = nullptr;  // device argument structs
    int* off = nullptr;    // device block offsets [n_cfg + 1] (params, finish)
    int4* blk = nullptr;   // device (cfg, phase, slab) per block (weights)
  };
  Launch params, weights[2], finish[4];
};
size_t table_batch_bytes(const TableBatchCfg* cfgs, int n_cfg);
// builds the work lists of cfgs (none with differential rotation) in d_buf
// (table_batch_bytes(n) bytes) and uploads them
hipError_t table_batch_upload(const TableBatchCfg* cfgs, int n, void* d_buf, TableBatch* tb);
// enqueues params, then weights, then finish (three dependent phases)
hipError_t table_batch_launch(const TableBatch& tb, hipStream_t st);
hipError_t launch_apply(soap_ctx* c, const Plan& pl, const void* d_win, const int* d_nvg, void* d_flux);
// apply with an explicit shape (threads per block, windows staged per LDS
// pass) on stream st
hipError_t launch_apply_shape(soap_ctx* c, const Plan& pl, const void* d_win, const int* d_nvg, void* d_flux,
                              int depth, int order, hipStream_t st);

// batched shift-and-sum: one launch over the (tile, chunk) items of many
// configurations of one precision and table mode (256-thread blocks)
struct ApplyBatchCfg {
  soap_ctx* c;
  Plan pl;
  const void* win;
  const int* nvg;
  void* flux;
};
struct ApplyBatchGroup {
  bool fp32 = true, paired = true;
  int n_cfg = 0, n_items = 0, depth = 2, order = 0, effect = SOAP_EFFECT_TOT, pc = 0;
  void* args = nullptr;  // device ApplyArgs[n_cfg]
  void* off = nullptr;   // device item offsets [n_cfg + 1]
};
size_t apply_batch_bytes(int n);
hipError_t apply_batch_upload(const ApplyBatchCfg* cfgs, int n, void* d_buf, ApplyBatchGroup* g);
hipError_t apply_batch_launch(const ApplyBatchGroup& g, hipStream_t st);
hipError_t launch_q_convert(soap_ctx* c, void* out);
// pads of `rows` padded rows starting at base (end samples held)
hipError_t launch_pad_rows(soap_ctx* c, void* base, int rows);
// sets *d_flag (device int, zeroed by the caller) when any of `rows` padded
// rows at base (float or double per the context) or, with Q set, the quiet
// spectrum holds a non-finite value
hipError_t launch_check_finite(soap_ctx* c, const void* base, int rows, bool with_q, int* d_flag);
// host tables of a mask (soap_ctx::ws_mask layout); false with err set when
// the velocity grid does not fit the kernel
bool ccf_build_tables(soap_ctx* c, const double* lnl, const double* wl, int nl, std::vector<unsigned char>& blob,
                      std::string& err);
// partial CCFs per line block, [n_lb][n_spec][n_v] in the flux type (a block's
// partial is a sum in that type)
hipError_t launch_ccf(soap_ctx* c, const void* d_flux, int64_t n_spec, int n_lines, void* d_part);
// a mask's CCF launch parameters (the context's layout of its tables, with
// the tables at `tables`), so that a batch can keep its own copy of them
struct CcfPlan {
  const unsigned char* tables = nullptr;
  size_t off_edges = 0, off_batch = 0, off_bfirst = 0;
  int npx = 2, stg = 256, nv = 0, n_lines = 0;
  double v0 = 0.0, dv = 0.0;
  bool fp32 = true;
  int64_t P = 0;
};
CcfPlan ccf_plan(const soap_ctx* c, int n_lines, const void* tables);
// One spectra set of a work-list CCF + fit launch (every set of one launch
// shares the mask layout: velocities, pixels per hole, stage width, float
// type).
struct CcfBatchSet {
  const void* flux;
  void* part;        // [nlb][n_spec][n_v] partials
  double* ccf;       // [n_spec][n_v]
  soap_rv* rv;       // [n_spec], or NULL (sums only)
  int64_t n_spec;
  int P, nlb;
  const unsigned char* tables;
  size_t off_edges, off_batch, off_bfirst;
};
struct CcfBatch {
  CcfPlan shape;               // a plan with the shared layout
  int n_sets = 0, n_ccf_blocks = 0, n_fit_blocks = 0;
  CcfBatchSet* sets = nullptr;  // device
  int4* ccf_blk = nullptr;      // device (set, line block, spectrum block)
  int2* fit_blk = nullptr;      // device (set, spectrum)
};
// same layout: the sets of one CcfBatch must agree on these
bool ccf_same_layout(const CcfPlan& a, const CcfPlan& b);
size_t ccf_batch_bytes(const CcfPlan* plans, const int64_t* n_spec, int n);
// sets i of plans[i] (tables, lines) and the given buffers; d_buf of
// ccf_batch_bytes bytes
hipError_t ccf_batch_upload(const CcfPlan* plans, const CcfBatchSet* sets, int n, void* d_buf, CcfBatch* cb);
hipError_t ccf_batch_launch(const CcfBatch& cb, hipStream_t st);
soap_status ctx_set_mask(soap_ctx* c, const soap_mask* mask);
hipError_t launch_ccf_p(const CcfPlan& q, hipStream_t st, const void* d_flux, int64_t n_spec, void* d_part);
hipError_t launch_ccf_fit_p(const CcfPlan& q, hipStream_t st, const void* d_part, int64_t n_spec, double* d_ccf,
                            soap_rv* d_rv);
// sums the partial CCFs (in double) into d_ccf and, when d_rv is not null,
// fits them
hipError_t launch_ccf_fit(soap_ctx* c, int n_lines, const void* d_part, int64_t n_spec, double* d_ccf,
                          soap_rv* d_rv);
hipError_t launch_ccf_linear_fit(soap_ctx* c, const float* d_coef, int64_t n, int k, const double* d_base,
                                 const double* d_basis, double* d_lin, double* d_ccf, soap_rv* d_rv);
hipError_t launch_sg_rv(soap_ctx* c, const float* d_coef, const float* d_members, int64_t n, int E, int k,
                        const double* d_base, const int* d_base_idx, int n_base, const double* d_basis,
                        double calib, double thr, soap_rv* d_rv, double* d_rv_kms, double* d_err,
                        int* d_fallback, void* d_work);
// device workspace of launch_sg_rv for n samples
size_t sg_rv_work_bytes(const soap_ctx* c, int64_t n);

// resolution lowering: kernel weights of a resolving power on the grid
// (false when the kernel would be wider than LSF_KMAX pixels each side), the
// largest spectrum count one launch takes, and the launch (in != out)
bool lsf_plan(double resolution, double dln, LsfPlan* pl);
int64_t lsf_max_spectra(int64_t P);
hipError_t launch_lsf(soap_ctx* c, const LsfPlan& pl, const void* in, void* out, int64_t n_spec, hipStream_t st);

// looks up this device's copy of the allocation-free entry point's scratch
// array (once per device; the device must be current); the result is kept
hipError_t scratch_setup(int device);

int ccf_line_blocks(int n_lines);
int ccf_span_pixels(bool fp32);

// true when `m` is the mask whose tables the context holds (set by the last
// soap_ccf_rv with a new mask)
inline bool mask_is_cached(const soap_ctx* c, const soap_mask* m) {
  const int nl = (int)m->n_lines;
  return c->mask_valid && m->n_lines == (int64_t)c->mask_lnl.size() && c->mask_h == m->half_width_kms &&
         c->mask_v0 == m->v0_kms && c->mask_dv == m->dv_kms && c->mask_nv == m->n_v && m->ln_lambda && m->weight &&
         std::memcmp(c->mask_lnl.data(), m->ln_lambda, sizeof(double) * nl) == 0 &&
         std::memcmp(c->mask_w.data(), m->weight, sizeof(double) * nl) == 0;
}

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

// index of the closest mu bin (ties to the lower index); mu_b is strictly
// decreasing, so the two candidates are found by bisection and compared
SOAP_DEV int nearest_bin(double mu, const double* mu_b, int B) {
#pragma clang fp contract(off)
  // first index with mu_b[idx] < mu (B if none)
  int lo = 0, hi = B;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (mu_b[mid] < mu) hi = mid;
    else lo = mid + 1;
  }
  if (lo == 0) return 0;
  if (lo == B) return B - 1;
  double da = fabs(mu - mu_b[lo - 1]);
  double db = fabs(mu - mu_b[lo]);
  return (db < da) ? lo : lo - 1;
}

// observer-frame unit vector of a region centre at a rotation phase; under
// differential rotation the region turns at its own latitude's rate,
// 1 + diff_rot sin^2(lat) equatorial turns per unit phase (exactly one for
// diff_rot = 0)
SOAP_DEV void region_centre(double lat, double lon, double phase, double incl, double diff_rot, double* cx,
                            double* cy, double* cz) {
#pragma clang fp contract(off)
  double th = lat * DEG;
  const double sl = sin(th);
  double psi = (lon + 360.0 * phase * (1.0 + diff_rot * sl * sl)) * DEG;
  double inc = incl * DEG;
  double X = cos(th) * sin(psi);
  double Y = sin(th);
  double Z = cos(th) * cos(psi);
  *cx = X;
  *cy = Y * sin(inc) - Z * cos(inc);
  *cz = Y * cos(inc) + Z * sin(inc);
}

// Shift of a cell in pixels and its interpolation split (Eqs. 6, 9-11 on
// the log grid): s = atanh(v / c) / dln with v = vsini x (1 + diff_rot
// sin^2 theta), sin theta = y sin i + mu cos i; the cell adds (1 - w) of its
// weight at offset ceil(s) and w at ceil(s) - 1, w = expm1(u dln) /
// expm1(dln), u = ceil(s) - s.
SOAP_DEV void cell_shift(double x, double y, double mu, double vsini, double diff_rot, double sin_i, double cos_i,
                         double dln, int* c, double* w) {
  const double st = y * sin_i + mu * cos_i;
  const double v = vsini * x * (1.0 + diff_rot * st * st);
  const double s = atanh(v / C_KMS) / dln;
  const double cc = ceil(s);
  *c = (int)cc;
  *w = expm1((cc - s) * dln) / expm1(dln);
}

}  // namespace soap
