// C ABI of libsoap (declarations and documentation in include/soap.h).
//
// This file holds argument validation, the context and its device workspace,
// host <-> device staging and the order of kernel launches.  All arithmetic of
// the method runs in the kernels of geom.hip, weights.hip, apply.hip and
// ccf.hip.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "soap_internal.hpp"

#define SOAP_API extern "C" __attribute__((visibility("default")))

namespace {

thread_local std::string g_init_err;

void setf(std::string& dst, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  dst = buf;
}

#define ARG_CHECK(cond, ...)        \
  do {                              \
    if (!(cond)) {                  \
      setf(err, __VA_ARGS__);       \
      return SOAP_ERR_ARG;          \
    }                               \
  } while (0)

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      const bool oom_ = e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation;  \
      setf(c->err, "%s failed: %s%s", #expr, hipGetErrorString(e_), oom_ ? soap::dev_cap_note() : ""); \
      return oom_ ? SOAP_ERR_OOM : SOAP_ERR_HIP;                                        \
    }                                                                                  \
  } while (0)

bool is_finite(double x) { return std::isfinite(x); }

template <typename T>
bool all_finite_host(const void* p, size_t n) {
  const T* a = static_cast<const T*>(p);
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite((double)a[i])) return false;
  return true;
}

soap_status validate_desc(const soap_star_desc* d, std::string& err) {
  ARG_CHECK(d != nullptr, "desc is NULL");
  ARG_CHECK(d->n_grid >= 2 && d->n_grid <= soap::MAX_GRID, "n_grid must be in [2, %d], got %d", soap::MAX_GRID,
            d->n_grid);
  ARG_CHECK(d->n_mu >= 1 && d->n_mu <= soap::MAX_MU, "n_mu must be in [1, %d], got %d", soap::MAX_MU, d->n_mu);
  ARG_CHECK(d->n_pix >= 8 && d->n_pix <= (int64_t(1) << 30), "n_pix must be in [8, 2^30], got %lld",
            (long long)d->n_pix);
  ARG_CHECK(d->precision == SOAP_PREC_FP32 || d->precision == SOAP_PREC_FP64, "unknown precision %d",
            d->precision);
  ARG_CHECK(d->contrast_mode == SOAP_CONTRAST_SCALAR || d->contrast_mode == SOAP_CONTRAST_PLANCK ||
                d->contrast_mode == SOAP_CONTRAST_ARRAY,
            "unknown contrast_mode %d", d->contrast_mode);
  ARG_CHECK(is_finite(d->vsini_kms) && std::fabs(d->vsini_kms) < 0.1 * soap::C_KMS, "vsini_kms out of range");
  ARG_CHECK(is_finite(d->incl_deg) && d->incl_deg >= 0.0 && d->incl_deg <= 180.0, "incl_deg must be in [0, 180]");
  ARG_CHECK(is_finite(d->ld_u1) && is_finite(d->ld_u2), "limb-darkening coefficients must be finite");
  ARG_CHECK(is_finite(d->diff_rot) && std::fabs(d->diff_rot) < 1.0, "diff_rot must be in (-1, 1)");
  ARG_CHECK(is_finite(d->ln_lambda0), "ln_lambda0 must be finite");
  ARG_CHECK(is_finite(d->dln_lambda) && d->dln_lambda > 0.0 && d->dln_lambda < 1.0, "dln_lambda must be in (0, 1)");
  ARG_CHECK(d->mu_bins != nullptr, "mu_bins is NULL");
  for (int b = 0; b < d->n_mu; ++b) {
    ARG_CHECK(is_finite(d->mu_bins[b]) && d->mu_bins[b] > 0.0 && d->mu_bins[b] <= 1.0,
              "mu_bins[%d] must be in (0, 1]", b);
    if (b) ARG_CHECK(d->mu_bins[b] < d->mu_bins[b - 1], "mu_bins must be strictly decreasing");
  }
  ARG_CHECK(d->spectra[SOAP_QUIET] != nullptr, "spectra[SOAP_QUIET] is NULL");
  if (!d->spectra_on_device) {
    const size_t n = (size_t)d->n_mu * (size_t)d->n_pix;
    for (int t = 0; t < 3; ++t) {
      if (!d->spectra[t]) continue;
      bool ok = (d->precision == SOAP_PREC_FP32) ? all_finite_host<float>(d->spectra[t], n)
                                                 : all_finite_host<double>(d->spectra[t], n);
      ARG_CHECK(ok, "spectra[%d] holds a non-finite value", t);
    }
  }
  if (d->contrast_mode == SOAP_CONTRAST_ARRAY) {
    ARG_CHECK(d->contrast[SOAP_QUIET] == nullptr, "contrast[SOAP_QUIET] must be NULL");
    for (int t = 1; t < 3; ++t) {
      ARG_CHECK(!d->spectra[t] || d->contrast[t], "contrast[%d] is required with spectra[%d]", t, t);
      if (d->contrast[t] && !d->spectra_on_device) {
        const size_t n = (size_t)d->n_mu * (size_t)d->n_pix;
        bool ok = (d->precision == SOAP_PREC_FP32) ? all_finite_host<float>(d->contrast[t], n)
                                                   : all_finite_host<double>(d->contrast[t], n);
        ARG_CHECK(ok, "contrast[%d] holds a non-finite value", t);
      }
    }
  } else {
    for (int t = 0; t < 3; ++t) ARG_CHECK(d->contrast[t] == nullptr, "contrast[%d] must be NULL outside ARRAY mode", t);
  }
  if (d->contrast_mode == SOAP_CONTRAST_PLANCK) {
    ARG_CHECK(is_finite(d->teff_k) && d->teff_k > 100.0, "teff_k must be > 100 K");
    ARG_CHECK(is_finite(d->dt_spot_k) && d->teff_k - d->dt_spot_k > 100.0, "spot temperature must be > 100 K");
    for (int b = 0; b < d->n_mu; ++b) {
      double mu = d->mu_bins[b];
      double dt = d->dt_fac_coef[0] + d->dt_fac_coef[1] * mu + d->dt_fac_coef[2] * mu * mu;
      ARG_CHECK(is_finite(dt) && d->teff_k + dt > 100.0, "facula temperature must be > 100 K");
    }
  }
  return SOAP_OK;
}

hipError_t grow(soap::Workspace& w, size_t bytes) {
  if (w.bytes >= bytes) return hipSuccess;
  if (w.ptr) {
    hipError_t e = soap::dev_free(w.ptr);
    if (e != hipSuccess) return e;
    w.ptr = nullptr;
    w.bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, 256);
  hipError_t e = soap::dev_malloc(&w.ptr, want);
  if (e == hipSuccess) w.bytes = want;
  return e;
}

void free_ws(soap::Workspace& w) {
  if (w.ptr) (void)soap::dev_free(w.ptr);
  w.ptr = nullptr;
  w.bytes = 0;
}

void destroy_ctx(soap_ctx* c) {
  if (!c) return;
  if (c->hip_used) {
    (void)hipStreamSynchronize(c->stream);
    if (c->side) (void)hipStreamSynchronize(c->side);
  }
  for (int t = 0; t < 3; ++t)
    if (c->d_spec_base[t]) (void)soap::dev_free(c->d_spec_base[t]);
  void* bufs[] = {c->d_mu, c->d_col_c, c->d_col_w, c->d_colW, c->d_Kq, c->d_Kq_fx, c->d_Q, c->d_con_base, c->d_ones};
  for (void* p : bufs)
    if (p) (void)soap::dev_free(p);
  soap::Workspace* ws[] = {&c->ws_flux, &c->ws_ccf, &c->ws_ccfout, &c->ws_rv, &c->ws_mask, &c->ws_specin,
                           &c->ws_lsf, &c->ws_sg};
  for (auto* w : ws) free_ws(*w);
  for (auto& S : c->prep) {
    soap::Workspace* pw[] = {&S.par, &S.Kfx, &S.K, &S.mask64, &S.vg, &S.nvg};
    for (auto* w : pw) free_ws(*w);
    if (S.prep_done) (void)hipEventDestroy(S.prep_done);
    if (S.apply_done) (void)hipEventDestroy(S.apply_done);
  }
  if (c->side) (void)hipStreamDestroy(c->side);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (int k = 0; k < soap_ctx::NSLOT; ++k) {
    if (c->slot[k]) (void)hipHostFree(c->slot[k]);
    if (c->slot_done[k]) (void)hipEventDestroy(c->slot_done[k]);
  }
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->pinned_done) (void)hipEventDestroy(c->pinned_done);
  delete c;
}

// copies n_rows rows of P samples (host or device) into padded device rows
// starting at dst; host rows go through pinned memory, so the copy is one
// DMA from memory that stays valid until it has completed
hipError_t upload_rows(soap_ctx* c, void* dst, const void* src, int n_rows, bool on_device) {
  const size_t row_bytes = (size_t)c->Pstride * c->esize;
  const size_t src_bytes = (size_t)c->P * c->esize * n_rows;
  void* pinned = nullptr;
  if (!on_device) {
    hipError_t e = hipHostMalloc(&pinned, src_bytes, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    std::memcpy(pinned, src, src_bytes);
    src = pinned;
  }
  hipError_t ce = hipMemcpy2DAsync(dst, row_bytes, src, (size_t)c->P * c->esize, (size_t)c->P * c->esize, n_rows,
                                   on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream);
  if (pinned) {
    const hipError_t se = hipStreamSynchronize(c->stream);
    (void)hipHostFree(pinned);
    if (ce == hipSuccess) ce = se;
  }
  return ce;
}

// sum over the visible cells of (2/N)^2 |I(mu)|: bounds every tap and
// column sum of the fixed-point accumulators
double disk_weight(int N, double u1, double u2) {
  const double area = (2.0 / N) * (2.0 / N);
  double tot = 0.0;
  for (int i = 0; i < N; ++i) {
    const double x = soap::cell_coord(i, N);
    for (int k = 0; k < N; ++k) {
      const double y = soap::cell_coord(k, N);
      const double r2 = x * x + y * y;
      if (r2 < 1.0) tot += area * std::fabs(soap::limb_dark(std::sqrt(1.0 - r2), u1, u2));
    }
  }
  return tot;
}

using soap::FX_RANGE;

soap_status init_impl(const soap_star_desc* d, soap_ctx* c) {
  c->N = d->n_grid;
  c->B = d->n_mu;
  c->P = d->n_pix;
  c->vsini = d->vsini_kms;
  c->incl = d->incl_deg;
  c->u1 = d->ld_u1;
  c->u2 = d->ld_u2;
  c->ln0 = d->ln_lambda0;
  c->dln = d->dln_lambda;
  c->diff_rot = d->diff_rot;
  c->sin_i = std::sin(c->incl * soap::DEG);
  c->cos_i = std::cos(c->incl * soap::DEG);
  c->prec = d->precision;
  c->cmode = d->contrast_mode;
  c->teff = d->teff_k;
  c->dt_spot = d->dt_spot_k;
  for (int i = 0; i < 3; ++i) c->dt_fac[i] = d->dt_fac_coef[i];
  c->mu_bins.assign(d->mu_bins, d->mu_bins + d->n_mu);
  c->esize = (c->prec == SOAP_PREC_FP32) ? sizeof(float) : sizeof(double);

  // tap offset range: a bound on the column shifts |s| <= atanh(|vsini| x_max / c) / dln
  // with one offset of margin on each side, so rounding of the device's
  // own shift can never leave the table
  // (differential rotation scales a cell's velocity by 1 + diff_rot sin^2,
  // at most max(1, 1 + diff_rot) in size)
  const double xmax = 1.0 - 1.0 / c->N;
  const double vscale = std::max(1.0, 1.0 + c->diff_rot);
  const double smax = std::atanh(std::fabs(c->vsini) * xmax * vscale / soap::C_KMS) / c->dln;
  c->jmin = -(int)std::floor(smax) - 2;
  c->jmax = (int)std::ceil(smax) + 1;
  c->J = c->jmax - c->jmin + 1;
  std::string& err = c->err;
  ARG_CHECK(c->J <= 64, "rotation shift of %.1f pixels exceeds the supported 30 pixels", smax);
  c->disk_weight = disk_weight(c->N, c->u1, c->u2);
  if (!(c->disk_weight < FX_RANGE)) {
    setf(c->err, "limb darkening gives a disk weight of %.3f, beyond the fixed-point range of the tap sums (%.2f)",
         c->disk_weight, FX_RANGE);
    return SOAP_ERR_UNSUPPORTED;
  }
  ARG_CHECK(c->P >= 2 * (int64_t)c->J + 4, "n_pix must be at least 2 * (max shift + 3) + 4");
  if (c->diff_rot != 0.0 && 3 * c->B * c->J > soap::DR_TAB_MAX) {
    setf(c->err, "differential rotation supports n_mu x shift range up to %d, got %d x %d", soap::DR_TAB_MAX / 3,
         c->B, c->J);
    return SOAP_ERR_UNSUPPORTED;
  }
  const size_t gj_bytes = (size_t)3 * c->B * c->J * sizeof(double) + 192 * sizeof(int);
  if (gj_bytes > 60 * 1024) {
    setf(c->err, "n_mu x shift range too large for the per-phase tap table (%zu bytes)", gj_bytes);
    return SOAP_ERR_UNSUPPORTED;
  }

  c->hip_used = true;
  HIP_TRY(hipGetDevice(&c->device));
  // the allocation-free entry point's scratch on this device (its status is
  // kept and reported by that entry point)
  (void)soap::scratch_setup(c->device);
  c->pc = (c->prec == SOAP_PREC_FP32) ? soap::PC_F32 : soap::PC_F64;
  c->n_tiles = (int)((c->P + soap::APPLY_TILE_MAX - 1) / soap::APPLY_TILE_MAX);
  // padded rows: PAD_FRONT samples before pixel 0, and past the last tile
  // enough room for the widest window the apply kernel reads
  const int64_t tail = (int64_t)c->n_tiles * soap::APPLY_TILE_MAX + 2 * soap::MAX_J + 64;
  c->Pstride = ((soap::PAD_FRONT + tail + 63) / 64) * 64;
  const size_t row_bytes = (size_t)c->Pstride * c->esize;
  const bool on_dev = d->spectra_on_device != 0;
  for (int t = 0; t < 3; ++t) {
    if (!d->spectra[t]) continue;
    HIP_TRY(soap::dev_malloc(&c->d_spec_base[t], row_bytes * c->B));
    c->d_spec[t] = static_cast<unsigned char*>(c->d_spec_base[t]) + soap::PAD_FRONT * c->esize;
    HIP_TRY(upload_rows(c, c->d_spec[t], d->spectra[t], c->B, on_dev));
    c->has_type[t] = true;
  }
  HIP_TRY(soap::dev_malloc((void**)&c->d_mu, sizeof(double) * c->B));
  HIP_TRY(hipMemcpy(c->d_mu, d->mu_bins, sizeof(double) * c->B, hipMemcpyHostToDevice));
  HIP_TRY(soap::dev_malloc((void**)&c->d_col_c, sizeof(int) * c->N));
  HIP_TRY(soap::dev_malloc((void**)&c->d_col_w, sizeof(double) * c->N));
  HIP_TRY(soap::dev_malloc((void**)&c->d_colW, sizeof(double) * c->N * c->B));
  HIP_TRY(soap::dev_malloc((void**)&c->d_Kq, sizeof(double) * c->B * c->J));
  if (c->diff_rot != 0.0) {
    HIP_TRY(soap::dev_malloc((void**)&c->d_Kq_fx, sizeof(unsigned long long) * c->B * c->J));
    HIP_TRY(hipMemsetAsync(c->d_Kq_fx, 0, sizeof(unsigned long long) * c->B * c->J, c->stream));
  }
  HIP_TRY(soap::dev_malloc((void**)&c->d_Q, sizeof(double) * c->n_tiles * soap::APPLY_TILE_MAX));
  HIP_TRY(soap::dev_malloc(&c->d_ones, c->esize * c->n_tiles * soap::APPLY_TILE_MAX));
  if (c->cmode == SOAP_CONTRAST_PLANCK) {
    // one spot row for every bin, one facula row per bin
    c->con_rows = c->B + 1;
    HIP_TRY(soap::dev_malloc(&c->d_con_base, row_bytes * c->con_rows));
    c->d_con_spot = static_cast<unsigned char*>(c->d_con_base) + soap::PAD_FRONT * c->esize;
    c->d_con_fac = static_cast<unsigned char*>(c->d_con_spot) + row_bytes;
    c->con_spot_stride = 0;
  } else if (c->cmode == SOAP_CONTRAST_ARRAY) {
    // the caller's rows: spot [B], then facula [B]; a type without spectra
    // keeps rows of zeros (never read)
    c->con_rows = 2 * c->B;
    HIP_TRY(soap::dev_malloc(&c->d_con_base, row_bytes * c->con_rows));
    c->d_con_spot = static_cast<unsigned char*>(c->d_con_base) + soap::PAD_FRONT * c->esize;
    c->d_con_fac = static_cast<unsigned char*>(c->d_con_spot) + row_bytes * c->B;
    c->con_spot_stride = c->Pstride;
    for (int t = 1; t < 3; ++t) {
      void* dst = t == SOAP_SPOT ? c->d_con_spot : c->d_con_fac;
      if (d->contrast[t]) HIP_TRY(upload_rows(c, dst, d->contrast[t], c->B, on_dev));
      else HIP_TRY(hipMemsetAsync(dst, 0, row_bytes * c->B - soap::PAD_FRONT * c->esize, c->stream));
    }
  }
  HIP_TRY(hipEventCreateWithFlags(&c->pinned_done, hipEventDisableTiming));
  for (int k = 0; k < soap_ctx::NSLOT; ++k) HIP_TRY(hipEventCreateWithFlags(&c->slot_done[k], hipEventDisableTiming));
  HIP_TRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  for (auto& S : c->prep) {
    HIP_TRY(hipEventCreateWithFlags(&S.prep_done, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&S.apply_done, hipEventDisableTiming));
  }

  HIP_TRY(soap::launch_pad(c));
  HIP_TRY(soap::launch_geom(c));
  HIP_TRY(soap::launch_ones(c));
  if (c->cmode == SOAP_CONTRAST_PLANCK) HIP_TRY(soap::launch_contrast(c));
  if (c->cmode == SOAP_CONTRAST_ARRAY) HIP_TRY(soap::launch_pad_rows(c, c->d_con_base, c->con_rows));
  HIP_TRY(soap::launch_quiet(c));
  // the device copies must be finite: device inputs were not checked on the
  // host, and a host input that was finite there yet is not here means the
  // upload went wrong
  // d_flag[0]: rows, d_flag[1]: quiet spectrum; read back with a blocking
  // copy once the stream is idle
  int* d_flag = nullptr;
  HIP_TRY(soap::dev_malloc((void**)&d_flag, 2 * sizeof(int)));
  int h_flag[2] = {0, 0};
  hipError_t fe = hipMemsetAsync(d_flag, 0, 2 * sizeof(int), c->stream);
  for (int t = 0; t < 3 && fe == hipSuccess; ++t)
    if (c->d_spec_base[t]) fe = soap::launch_check_finite(c, c->d_spec_base[t], c->B, false, d_flag);
  if (fe == hipSuccess && c->d_con_base) fe = soap::launch_check_finite(c, c->d_con_base, c->con_rows, false, d_flag);
  if (fe == hipSuccess) fe = soap::launch_check_finite(c, nullptr, 0, true, d_flag + 1);
  // host arrays (mu bins, spectra) may be released once the call returns
  const hipError_t se = hipStreamSynchronize(c->stream);
  const hipError_t me =
      (fe == hipSuccess && se == hipSuccess) ? hipMemcpy(h_flag, d_flag, sizeof h_flag, hipMemcpyDeviceToHost) : fe;
  (void)soap::dev_free(d_flag);
  HIP_TRY(fe);
  HIP_TRY(se);
  HIP_TRY(me);
  if (h_flag[0] || h_flag[1]) {
    const char* what = h_flag[0] ? "the device copy of the local spectra or contrast arrays"
                                 : "the quiet integrated spectrum";
    if (on_dev) {
      setf(c->err, "%s holds a non-finite value (device inputs)", what);
      return SOAP_ERR_ARG;
    }
    setf(c->err, "%s holds a non-finite value although the host inputs are finite: the upload failed", what);
    return SOAP_ERR_HIP;
  }
  return SOAP_OK;
}

// copy a small host block to device memory through pinned staging; the host
// waits for the previous staging copy before overwriting the buffer
soap_status stage_to_device(soap_ctx* c, const void* src, size_t bytes, void* dst) {
  if (c->pinned_bytes < bytes) {
    HIP_TRY(hipEventSynchronize(c->pinned_done));
    if (c->pinned) HIP_TRY(hipHostFree(c->pinned));
    c->pinned = nullptr;
    c->pinned_bytes = 0;
    size_t want = std::max<size_t>(bytes, 64 * 1024);
    HIP_TRY(hipHostMalloc(&c->pinned, want, hipHostMallocDefault));
    c->pinned_bytes = want;
  } else {
    HIP_TRY(hipEventSynchronize(c->pinned_done));
  }
  std::memcpy(c->pinned, src, bytes);
  HIP_TRY(hipMemcpyAsync(dst, c->pinned, bytes, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipEventRecord(c->pinned_done, c->stream));
  return SOAP_OK;
}

const char* const kStageName[] = {"soap:weights", "soap:compact", "soap:apply", "soap:ccf", "soap:fit", "soap:lsf"};

// Brackets one stage with events on the context stream when profiling is on,
// and always with a roctx range named after the stage (the host-side span of
// its enqueue, seen by a marker trace).
struct StageTimer {
  soap_ctx* c;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  bool open = true;
  StageTimer(soap_ctx* c_, int s, hipStream_t st_ = nullptr) : c(c_), stage(s), st(st_ ? st_ : c_->stream) {
    roctxRangePushA(kStageName[s]);
    if (c->prof && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, st);
  }
  ~StageTimer() {
    if (open) roctxRangePop();
  }
  void done() {
    if (open) roctxRangePop();
    open = false;
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, st) == hipSuccess) {
      c->pending.push_back({stage, a, b});
    } else {
      (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
    a = nullptr;
  }
};

enum { ST_WEIGHTS = 0, ST_COMPACT = 1, ST_APPLY = 2, ST_CCF = 3, ST_GFIT = 4, ST_LSF = 5 };

}  // namespace

SOAP_API int32_t soap_abi_version(void) { return SOAP_ABI_VERSION; }

SOAP_API uint64_t soap_device_bytes(void) { return soap::dev_bytes_held(); }

SOAP_API const char* soap_status_string(soap_status s) {
  switch (s) {
    case SOAP_OK: return "SOAP_OK";
    case SOAP_ERR_ARG: return "SOAP_ERR_ARG";
    case SOAP_ERR_OOM: return "SOAP_ERR_OOM";
    case SOAP_ERR_HIP: return "SOAP_ERR_HIP";
    case SOAP_ERR_STATE: return "SOAP_ERR_STATE";
    case SOAP_ERR_NOCONV: return "SOAP_ERR_NOCONV";
    case SOAP_ERR_UNSUPPORTED: return "SOAP_ERR_UNSUPPORTED";
  }
  return "unknown soap_status";
}

SOAP_API const char* soap_last_error(const soap_ctx* c) {
  if (!c) return g_init_err.c_str();
  return c->err.c_str();
}

SOAP_API soap_status soap_grid_init(const soap_star_desc* desc, void* hip_stream, soap_ctx** out) {
  if (!out) {
    g_init_err = "out is NULL";
    return SOAP_ERR_ARG;
  }
  *out = nullptr;
  {
    std::string err;
    soap_status st = validate_desc(desc, err);
    if (st != SOAP_OK) {
      g_init_err = err;
      return st;
    }
  }
  soap_ctx* c = new (std::nothrow) soap_ctx();
  if (!c) {
    g_init_err = "host allocation of the context failed";
    return SOAP_ERR_OOM;
  }
  c->stream = static_cast<hipStream_t>(hip_stream);
  soap_status st = init_impl(desc, c);
  if (st != SOAP_OK) {
    g_init_err = c->err;
    destroy_ctx(c);
    return st;
  }
  *out = c;
  return SOAP_OK;
}

SOAP_API soap_status soap_quiet_spectrum(soap_ctx* c, void* out, int32_t out_on_device) {
  if (!c) return SOAP_ERR_ARG;
  std::string& err = c->err;
  ARG_CHECK(out != nullptr, "out is NULL");
  const size_t bytes = (size_t)c->P * c->esize;
  void* dst = out;
  if (!out_on_device) {
    HIP_TRY(grow(c->ws_flux, bytes));
    dst = c->ws_flux.ptr;
  }
  if (c->prec == SOAP_PREC_FP64)
    HIP_TRY(hipMemcpyAsync(dst, c->d_Q, bytes, hipMemcpyDeviceToDevice, c->stream));
  else
    HIP_TRY(soap::launch_q_convert(c, dst));
  if (!out_on_device) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(out, dst, bytes, hipMemcpyDeviceToHost));
  }
  return SOAP_OK;
}

namespace {

// Shared body of soap_active_spectra and soap_active_spectra_jobs.  With
// pj_host == NULL every phase uses regions[0 .. n_regions); otherwise phase
// p uses pj_host[p] = (first region, count).  Arguments are validated.
soap_status active_impl(soap_ctx* c, const soap_region* regions, int32_t n_regions, int max_reg,
                        const int2* pj_host, const double* phases, int32_t n_phases, int32_t effect, void* flux,
                        int32_t flux_on_device) {
  // per-call plan: paired tables when every active weight equals its
  // removal weight (chromatic contrast, the convective effect, or unit
  // scalar contrasts); otherwise split tables with explicit removal rows
  soap::Plan pl;
  pl.n_ph = n_phases;
  pl.effect = effect;
  bool unit = true;
  for (int r = 0; r < n_regions; ++r) unit = unit && regions[r].contrast == 1.0;
  pl.paired = (c->cmode != SOAP_CONTRAST_SCALAR || effect == SOAP_EFFECT_BCONV || unit) ? 1 : 0;
  if (!pl.paired) {
    // split tables scale the active rows by the region contrasts
    double cmax = 1.0;
    for (int r = 0; r < n_regions; ++r) cmax = std::max(cmax, regions[r].contrast);
    if (!(c->disk_weight * cmax < FX_RANGE)) {
      setf(c->err, "disk weight %.3f x contrast %.3f reaches the fixed-point range of the tap sums (%.2f)",
           c->disk_weight, cmax, FX_RANGE);
      return SOAP_ERR_UNSUPPORTED;
    }
  }
  pl.G = (pl.paired ? 2 : 3) * c->B;
  pl.n_slabs = (c->N + soap::SLAB_COLS - 1) / soap::SLAB_COLS;
  pl.pc = c->pc;
  pl.n_chunks = (n_phases + pl.pc - 1) / pl.pc;
  pl.vg_cap = pl.G * ((c->J + soap::APPLY_JW - 1) / soap::APPLY_JW);
  const size_t GJ = (size_t)pl.G * c->J;

  // parameter block (regions then phases) in the next pinned slot; the
  // weights kernel reads it in place
  const size_t n_reg_slots = std::max<size_t>(soap::MAX_REGIONS, (size_t)n_regions);
  const size_t reg_bytes = 256 * ((sizeof(soap::Region) * n_reg_slots + 255) / 256);
  const size_t ph_bytes = 256 * ((sizeof(double) * n_phases + 255) / 256);
  const size_t par_bytes = reg_bytes + ph_bytes + (pj_host ? sizeof(int2) * n_phases : 0);
  // this call's table set; its kernels run on the side stream after the
  // apply that last read the set (two calls ago) is done
  const int sidx = c->prep_next;
  soap_ctx::PrepSet& S = c->prep[sidx];
  c->prep_next ^= 1;
  const size_t reg_dev = reg_bytes;
  const size_t pj_dev = 256 * ((sizeof(int2) * (size_t)n_phases + 255) / 256);
  const size_t cen_dev = 256 * ((sizeof(double4) * (size_t)n_phases * std::max(1, max_reg) + 255) / 256);
  const size_t par_dev = reg_dev + pj_dev + cen_dev + sizeof(int4) * (size_t)n_phases;
  const size_t kfx_bytes = sizeof(unsigned long long) * (size_t)n_phases * GJ;
  const size_t k_bytes = sizeof(double) * (size_t)n_phases * GJ;
  const size_t m_bytes = sizeof(unsigned long long) * (size_t)n_phases * pl.G;
  const size_t vg_bytes = (size_t)soap::win_bytes(pl.pc, (int)c->esize) * pl.n_chunks * pl.vg_cap;
  const size_t nvg_bytes = sizeof(int) * (size_t)pl.n_chunks;
  const bool regrow = S.par.bytes < par_dev || S.Kfx.bytes < kfx_bytes || S.K.bytes < k_bytes ||
                      S.mask64.bytes < m_bytes || S.vg.bytes < vg_bytes || S.nvg.bytes < nvg_bytes;
  if (regrow) {
    // buffers are replaced only with both streams idle
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipStreamSynchronize(c->side));
    HIP_TRY(grow(S.par, par_dev));
    HIP_TRY(grow(S.K, k_bytes));
    HIP_TRY(grow(S.mask64, m_bytes));
    HIP_TRY(grow(S.vg, vg_bytes));
    HIP_TRY(grow(S.nvg, nvg_bytes));
  }
  HIP_TRY(hipStreamWaitEvent(c->side, S.apply_done, 0));
  if (S.Kfx.bytes < kfx_bytes || S.kfx_dirty) {
    // fixed-point tap accumulators: zero when allocated; every call that
    // accumulates also clears them, so they are zeroed again only after an
    // interrupted call
    HIP_TRY(grow(S.Kfx, kfx_bytes));
    HIP_TRY(hipMemsetAsync(S.Kfx.ptr, 0, S.Kfx.bytes, c->side));
    S.kfx_dirty = false;
  }
  const size_t out_bytes = (size_t)n_phases * c->P * c->esize;
  void* dflux = flux;
  if (!flux_on_device) {
    HIP_TRY(grow(c->ws_flux, out_bytes));
    dflux = c->ws_flux.ptr;
  }
  // with resolution lowering the synthesis goes to a workspace first
  void* dsyn = dflux;
  const bool lower = c->lsf_resolution > 0.0;
  if (lower && n_phases > soap::lsf_max_spectra(c->P)) {
    setf(c->err, "resolution lowering takes at most %lld spectra per call", (long long)soap::lsf_max_spectra(c->P));
    return SOAP_ERR_UNSUPPORTED;
  }
  if (lower) {
    if (c->ws_lsf.bytes < out_bytes) {
      HIP_TRY(hipStreamSynchronize(c->stream));
      HIP_TRY(grow(c->ws_lsf, out_bytes));
    }
    dsyn = c->ws_lsf.ptr;
  }
  const int k = c->slot_next;
  c->slot_next = (k + 1) % soap_ctx::NSLOT;
  HIP_TRY(hipEventSynchronize(c->slot_done[k]));
  if (c->slot_bytes[k] < par_bytes) {
    if (c->slot[k]) HIP_TRY(hipHostFree(c->slot[k]));
    c->slot[k] = nullptr;
    c->slot_bytes[k] = 0;
    const size_t want = std::max<size_t>(par_bytes, 16 * 1024);
    HIP_TRY(hipHostMalloc(&c->slot[k], want, hipHostMallocMapped | hipHostMallocCoherent));
    c->slot_bytes[k] = want;
  }
  unsigned char* host = static_cast<unsigned char*>(c->slot[k]);
  soap::Region* hr = reinterpret_cast<soap::Region*>(host);
  for (int r = 0; r < n_regions; ++r) {
    hr[r].type = regions[r].type;
    hr[r].pad = 0;
    hr[r].lat_deg = regions[r].lat_deg;
    hr[r].lon_deg = regions[r].lon_deg;
    hr[r].radius = regions[r].radius;
    hr[r].contrast = regions[r].contrast;
  }
  std::memcpy(host + reg_bytes, phases, sizeof(double) * n_phases);
  if (pj_host) std::memcpy(host + reg_bytes + ph_bytes, pj_host, sizeof(int2) * n_phases);
  void* dev_view = nullptr;
  HIP_TRY(hipHostGetDevicePointer(&dev_view, c->slot[k], 0));
  const soap::Region* d_reg = static_cast<const soap::Region*>(dev_view);
  const double* d_ph = reinterpret_cast<const double*>(static_cast<const unsigned char*>(dev_view) + reg_bytes);
  const int2* d_pj =
      pj_host ? reinterpret_cast<const int2*>(static_cast<const unsigned char*>(dev_view) + reg_bytes + ph_bytes)
              : nullptr;

  soap::WeightsOut wo;
  wo.reg = static_cast<soap::Region*>(S.par.ptr);
  wo.pj = reinterpret_cast<int2*>(static_cast<unsigned char*>(S.par.ptr) + reg_dev);
  wo.cen = reinterpret_cast<double4*>(static_cast<unsigned char*>(S.par.ptr) + reg_dev + pj_dev);
  wo.box = reinterpret_cast<int4*>(static_cast<unsigned char*>(S.par.ptr) + reg_dev + pj_dev + cen_dev);
  wo.Kfx = static_cast<unsigned long long*>(S.Kfx.ptr);
  wo.K = static_cast<double*>(S.K.ptr);
  wo.mask = static_cast<unsigned long long*>(S.mask64.ptr);
  wo.wins = static_cast<unsigned char*>(S.vg.ptr);
  wo.nvg = static_cast<int*>(S.nvg.ptr);
  S.kfx_dirty = true;
  {
    StageTimer t(c, ST_WEIGHTS, c->side);
    HIP_TRY(soap::launch_weights(c, pl, d_reg, n_regions, std::max(1, max_reg), d_ph, d_pj, wo, c->side));
    t.done();
  }
  HIP_TRY(hipEventRecord(c->slot_done[k], c->side));
  {
    StageTimer t(c, ST_COMPACT, c->side);
    HIP_TRY(soap::launch_finish(c, pl, wo, c->side));
    t.done();
  }
  S.kfx_dirty = false;
  HIP_TRY(hipEventRecord(S.prep_done, c->side));
  HIP_TRY(hipStreamWaitEvent(c->stream, S.prep_done, 0));
  {
    StageTimer t(c, ST_APPLY);
    HIP_TRY(soap::launch_apply(c, pl, S.vg.ptr, static_cast<const int*>(S.nvg.ptr), dsyn));
    t.done();
  }
  HIP_TRY(hipEventRecord(S.apply_done, c->stream));
  if (lower) {
    StageTimer t(c, ST_LSF);
    HIP_TRY(soap::launch_lsf(c, c->lsf, dsyn, dflux, n_phases, c->stream));
    t.done();
  }
  c->last_prep = sidx;
  c->active_calls++;
  c->last_phases = n_phases;
  c->last_effect = effect;
  c->last_vg_cap = pl.vg_cap;
  c->last_pc = pl.pc;
  c->last_paired = pl.paired;
  if (dflux != flux) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(flux, dflux, out_bytes, hipMemcpyDeviceToHost));
  }
  return SOAP_OK;
}

soap_status check_region(soap_ctx* c, const soap_region& R, int r, int32_t effect) {
  std::string& err = c->err;
  ARG_CHECK(R.type == SOAP_SPOT || R.type == SOAP_FACULA, "regions[%d].type must be SOAP_SPOT or SOAP_FACULA", r);
  ARG_CHECK(is_finite(R.lat_deg) && R.lat_deg >= -90.0 && R.lat_deg <= 90.0, "regions[%d].lat_deg out of range", r);
  ARG_CHECK(is_finite(R.lon_deg), "regions[%d].lon_deg is not finite", r);
  ARG_CHECK(is_finite(R.radius) && R.radius > 0.0 && R.radius < 1.0, "regions[%d].radius must be in (0, 1)", r);
  ARG_CHECK(is_finite(R.contrast) && R.contrast > 0.0, "regions[%d].contrast must be > 0", r);
  if (effect != SOAP_EFFECT_FLUX)
    ARG_CHECK(c->has_type[R.type], "regions[%d] has type %d but the star has no spectra of that type", r, R.type);
  return SOAP_OK;
}

soap_status check_common(soap_ctx* c, const double* phases, int64_t n_phases, int32_t effect, void* flux) {
  std::string& err = c->err;
  ARG_CHECK(n_phases >= 1 && n_phases <= soap::MAX_PHASES, "n_phases must be in [1, %d]", soap::MAX_PHASES);
  ARG_CHECK(phases != nullptr, "phases is NULL");
  ARG_CHECK(effect == SOAP_EFFECT_TOT || effect == SOAP_EFFECT_FLUX || effect == SOAP_EFFECT_BCONV,
            "unknown effect %d", effect);
  ARG_CHECK(flux != nullptr, "flux is NULL");
  for (int64_t p = 0; p < n_phases; ++p) ARG_CHECK(is_finite(phases[p]), "phases[%lld] is not finite", (long long)p);
  return SOAP_OK;
}

}  // namespace

SOAP_API soap_status soap_active_spectra(soap_ctx* c, const soap_region* regions, int32_t n_regions,
                                         const double* phases, int32_t n_phases, int32_t effect, void* flux,
                                         int32_t flux_on_device) {
  if (!c) return SOAP_ERR_ARG;
  std::string& err = c->err;
  ARG_CHECK(n_regions >= 0 && n_regions <= soap::MAX_REGIONS, "n_regions must be in [0, %d]", soap::MAX_REGIONS);
  ARG_CHECK(n_regions == 0 || regions != nullptr, "regions is NULL");
  soap_status st = check_common(c, phases, n_phases, effect, flux);
  if (st != SOAP_OK) return st;
  for (int r = 0; r < n_regions; ++r)
    if ((st = check_region(c, regions[r], r, effect)) != SOAP_OK) return st;
  return active_impl(c, regions, n_regions, n_regions, nullptr, phases, n_phases, effect, flux, flux_on_device);
}

SOAP_API soap_status soap_active_spectra_jobs(soap_ctx* c, const soap_region* regions,
                                              const int32_t* region_offsets, const double* phases,
                                              const int32_t* phase_offsets, int32_t n_jobs, int32_t effect,
                                              void* flux, int32_t flux_on_device) {
  if (!c) return SOAP_ERR_ARG;
  std::string& err = c->err;
  ARG_CHECK(n_jobs >= 1 && n_jobs <= soap::MAX_PHASES, "n_jobs must be in [1, %d]", soap::MAX_PHASES);
  ARG_CHECK(region_offsets && phase_offsets, "offset arrays are NULL");
  ARG_CHECK(region_offsets[0] == 0 && phase_offsets[0] == 0, "offsets must start at 0");
  int max_reg = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const int64_t nr = (int64_t)region_offsets[j + 1] - region_offsets[j];
    const int64_t np = (int64_t)phase_offsets[j + 1] - phase_offsets[j];
    ARG_CHECK(nr >= 0 && nr <= soap::MAX_REGIONS, "job %d has %lld regions (0 .. %d allowed)", j, (long long)nr,
              soap::MAX_REGIONS);
    ARG_CHECK(np >= 1, "job %d has no phases", j);
    max_reg = std::max(max_reg, (int)nr);
  }
  const int64_t n_regions = region_offsets[n_jobs], n_phases = phase_offsets[n_jobs];
  ARG_CHECK(n_regions <= (int64_t(1) << 22), "at most 2^22 regions in all");
  ARG_CHECK(n_regions == 0 || regions != nullptr, "regions is NULL");
  soap_status st = check_common(c, phases, n_phases, effect, flux);
  if (st != SOAP_OK) return st;
  for (int64_t r = 0; r < n_regions; ++r)
    if ((st = check_region(c, regions[r], (int)r, effect)) != SOAP_OK) return st;
  std::vector<int2> pj((size_t)n_phases);
  for (int j = 0; j < n_jobs; ++j)
    for (int p = phase_offsets[j]; p < phase_offsets[j + 1]; ++p)
      pj[p] = make_int2(region_offsets[j], region_offsets[j + 1] - region_offsets[j]);
  return active_impl(c, regions, (int32_t)n_regions, max_reg, pj.data(), phases, (int32_t)n_phases, effect, flux,
                     flux_on_device);
}

namespace {

bool law_ok(const soap_evolution& e) {
  if (!is_finite(e.t0_days) || !is_finite(e.size0_msh) || !(e.size0_msh > 0.0) || !(e.size0_msh < 1e6)) return false;
  switch (e.mode) {
    case SOAP_EVOLVE_NONE: return true;
    case SOAP_EVOLVE_LINEAR_GROWTH:
    case SOAP_EVOLVE_LINEAR_DECAY: return is_finite(e.rate_msh_day) && e.rate_msh_day >= 0.0;
    case SOAP_EVOLVE_ASYM_GAUSS:
      return is_finite(e.fwhm_days) && e.fwhm_days > 0.0 && is_finite(e.asym_per_day);
  }
  return false;
}

double law_size(const soap_evolution& e, double t) {
  const double d = t - e.t0_days;
  switch (e.mode) {
    case SOAP_EVOLVE_LINEAR_GROWTH: return d >= 0.0 ? e.size0_msh + e.rate_msh_day * d : e.size0_msh;
    case SOAP_EVOLVE_LINEAR_DECAY: return d >= 0.0 ? std::max(0.0, e.size0_msh - e.rate_msh_day * d) : e.size0_msh;
    case SOAP_EVOLVE_ASYM_GAUSS: {
      const double sigma = e.fwhm_days / (2.0 * std::sqrt(2.0 * std::log(2.0)));
      const double w = sigma * (1.0 + e.asym_per_day * d);
      return w > 0.0 ? e.size0_msh * std::exp(-(d * d) / (2.0 * w * w)) : 0.0;
    }
    default: return e.size0_msh;
  }
}

}  // namespace

SOAP_API double soap_evolution_size(const soap_evolution* law, double t_days) {
  if (!law || !law_ok(*law) || !is_finite(t_days)) return std::nan("");
  return law_size(*law, t_days);
}

SOAP_API soap_status soap_active_spectra_evolving(soap_ctx* c, const soap_region* regions,
                                                  const soap_evolution* laws, int32_t n_regions,
                                                  const double* phases, int32_t n_phases, double prot_days,
                                                  int32_t effect, void* flux, int32_t flux_on_device) {
  if (!c) return SOAP_ERR_ARG;
  std::string& err = c->err;
  ARG_CHECK(n_regions >= 0 && n_regions <= soap::MAX_REGIONS, "n_regions must be in [0, %d]", soap::MAX_REGIONS);
  ARG_CHECK(n_regions == 0 || (regions != nullptr && laws != nullptr), "regions or laws is NULL");
  ARG_CHECK(is_finite(prot_days) && prot_days > 0.0, "prot_days must be > 0");
  soap_status st = check_common(c, phases, n_phases, effect, flux);
  if (st != SOAP_OK) return st;
  for (int r = 0; r < n_regions; ++r) {
    ARG_CHECK(law_ok(laws[r]), "laws[%d] is invalid (mode, size0 in (0, 1e6), rate >= 0, fwhm > 0)", r);
    soap_region probe = regions[r];
    probe.radius = 0.5;  // the radius comes from the law
    if ((st = check_region(c, probe, r, effect)) != SOAP_OK) return st;
  }
  // per-phase region lists: the regions of non-zero size with their radii
  std::vector<soap_region> flat;
  flat.reserve((size_t)n_regions * n_phases);
  std::vector<int2> pj((size_t)n_phases);
  int max_reg = 0;
  for (int p = 0; p < n_phases; ++p) {
    const double t = phases[p] * prot_days;
    const int first = (int)flat.size();
    for (int r = 0; r < n_regions; ++r) {
      const double a = law_size(laws[r], t);
      if (!(a > 0.0)) continue;
      const double f = std::min(1.0, a * 1e-6);
      soap_region g = regions[r];
      g.radius = std::sqrt(f * (2.0 - f));
      ARG_CHECK(g.radius < 1.0, "region %d reaches the whole hemisphere at phase %d", r, p);
      flat.push_back(g);
    }
    pj[p] = make_int2(first, (int)flat.size() - first);
    max_reg = std::max(max_reg, pj[p].y);
  }
  ARG_CHECK(flat.size() <= (size_t(1) << 22), "at most 2^22 regions over all phases");
  return active_impl(c, flat.empty() ? regions : flat.data(), (int32_t)flat.size(), max_reg, pj.data(), phases,
                     n_phases, effect, flux, flux_on_device);
}

SOAP_API soap_status soap_set_instrument(soap_ctx* c, double resolution) {
  if (!c) return SOAP_ERR_ARG;
  std::string& err = c->err;
  ARG_CHECK(is_finite(resolution) && resolution >= 0.0, "resolution must be >= 0");
  if (resolution == 0.0) {
    c->lsf_resolution = 0.0;
    return SOAP_OK;
  }
  soap::LsfPlan pl;
  if (!soap::lsf_plan(resolution, c->dln, &pl)) {
    setf(c->err, "resolution %.6g gives a line-spread function wider than %d pixels each side", resolution,
         soap::LSF_KMAX);
    return SOAP_ERR_UNSUPPORTED;
  }
  c->lsf = pl;
  c->lsf_resolution = resolution;
  return SOAP_OK;
}

SOAP_API soap_status soap_instrument_lsf(soap_ctx* c, const void* in, void* out, int64_t n_spec, double resolution,
                                         int32_t on_device) {
  if (!c) return SOAP_ERR_ARG;
  std::string& err = c->err;
  ARG_CHECK(in != nullptr && out != nullptr, "in or out is NULL");
  ARG_CHECK(n_spec >= 1 && n_spec <= soap::lsf_max_spectra(c->P), "n_spec must be in [1, %lld]",
            (long long)soap::lsf_max_spectra(c->P));
  ARG_CHECK(is_finite(resolution) && resolution > 0.0, "resolution must be > 0");
  const size_t bytes = (size_t)n_spec * c->P * c->esize;
  const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
  ARG_CHECK(a + bytes <= b || b + bytes <= a, "in and out overlap");
  soap::LsfPlan pl;
  if (!soap::lsf_plan(resolution, c->dln, &pl)) {
    setf(c->err, "resolution %.6g gives a line-spread function wider than %d pixels each side", resolution,
         soap::LSF_KMAX);
    return SOAP_ERR_UNSUPPORTED;
  }
  const void* din = in;
  void* dout = out;
  if (!on_device) {
    HIP_TRY(grow(c->ws_specin, bytes));
    soap_status st = stage_to_device(c, in, bytes, c->ws_specin.ptr);
    if (st != SOAP_OK) return st;
    din = c->ws_specin.ptr;
    HIP_TRY(grow(c->ws_lsf, bytes));
    dout = c->ws_lsf.ptr;
  }
  {
    StageTimer t(c, ST_LSF);
    HIP_TRY(soap::launch_lsf(c, pl, din, dout, n_spec, c->stream));
    t.done();
  }
  if (!on_device) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(out, dout, bytes, hipMemcpyDeviceToHost));
  }
  return SOAP_OK;
}

namespace soap {

// Validates a mask for the context and uploads its CCF tables unless they are
// the cached ones (soap_ccf_rv, batches with a CCF stage).
soap_status ctx_set_mask(soap_ctx* c, const soap_mask* mask) {
  std::string& err = c->err;
  ARG_CHECK(mask != nullptr, "mask is NULL");
  ARG_CHECK(mask->n_lines >= 1 && mask->n_lines <= (int64_t(1) << 20), "mask.n_lines must be in [1, 2^20]");
  ARG_CHECK(mask->ln_lambda != nullptr && mask->weight != nullptr, "mask arrays are NULL");
  ARG_CHECK(mask->n_v >= 4 && mask->n_v <= 768, "mask.n_v must be in [4, 768]");
  ARG_CHECK(is_finite(mask->v0_kms) && is_finite(mask->dv_kms) && mask->dv_kms > 0.0, "mask velocity grid invalid");
  ARG_CHECK(is_finite(mask->half_width_kms) && mask->half_width_kms > 0.0, "mask.half_width_kms must be > 0");
  const double vlo = mask->v0_kms - mask->half_width_kms;
  const double vhi = mask->v0_kms + mask->dv_kms * (mask->n_v - 1) + mask->half_width_kms;
  ARG_CHECK(std::fabs(vlo) < 0.1 * soap::C_KMS && std::fabs(vhi) < 0.1 * soap::C_KMS,
            "mask velocity grid beyond 0.1 c");
  const double hole_px = 2.0 * std::atanh(mask->half_width_kms / soap::C_KMS) / c->dln;
  if (hole_px > 8.0) {
    setf(c->err, "mask holes of %.2f pixels exceed the supported 8 pixels", hole_px);
    return SOAP_ERR_UNSUPPORTED;
  }
  const double reach_px = (std::atanh(vhi / soap::C_KMS) - std::atanh(vlo / soap::C_KMS)) / c->dln;
  if (reach_px + 4.0 > soap::ccf_span_pixels(c->prec == SOAP_PREC_FP32)) {
    setf(c->err, "the velocity grid spans %.0f pixels, beyond the supported %d", reach_px,
         soap::ccf_span_pixels(c->prec == SOAP_PREC_FP32) - 4);
    return SOAP_ERR_UNSUPPORTED;
  }
  const int nl = (int)mask->n_lines;
  for (int l = 0; l < nl; ++l)
    ARG_CHECK(is_finite(mask->ln_lambda[l]) && is_finite(mask->weight[l]), "mask line %d is not finite", l);

  // mask upload when it differs from the cached one
  const bool same = soap::mask_is_cached(c, mask);
  if (!same) {
    c->mask_valid = false;
    c->mask_h = mask->half_width_kms;
    c->mask_v0 = mask->v0_kms;
    c->mask_dv = mask->dv_kms;
    c->mask_nv = mask->n_v;
    std::vector<unsigned char> blob;
    std::string terr;
    if (!soap::ccf_build_tables(c, mask->ln_lambda, mask->weight, nl, blob, terr)) {
      c->err = terr;
      return SOAP_ERR_UNSUPPORTED;
    }
    HIP_TRY(grow(c->ws_mask, blob.size()));
    c->mask_blob_bytes = blob.size();
    soap_status st = stage_to_device(c, blob.data(), blob.size(), c->ws_mask.ptr);
    if (st != SOAP_OK) return st;
    c->mask_lnl.assign(mask->ln_lambda, mask->ln_lambda + nl);
    c->mask_w.assign(mask->weight, mask->weight + nl);
    c->mask_valid = true;
  }

  return SOAP_OK;
}

}  // namespace soap

SOAP_API soap_status soap_ccf_rv(soap_ctx* c, const void* flux, int32_t flux_on_device, int64_t n_spec,
                                 const soap_mask* mask, double* ccf_out, int32_t ccf_on_device, soap_rv* rv_out,
                                 int32_t rv_on_device) {
  if (!c) return SOAP_ERR_ARG;
  std::string& err = c->err;
  ARG_CHECK(flux != nullptr, "flux is NULL");
  ARG_CHECK(n_spec >= 1 && n_spec <= (int64_t(1) << 24), "n_spec must be in [1, 2^24]");
  {
    const soap_status ms = soap::ctx_set_mask(c, mask);
    if (ms != SOAP_OK) return ms;
  }
  const int nl = c->ccf_nl;  // the lines in the tables

  const void* dflux = flux;
  const size_t in_bytes = (size_t)n_spec * c->P * c->esize;
  if (!flux_on_device) {
    HIP_TRY(grow(c->ws_specin, in_bytes));
    // through the context's pinned staging, not an asynchronous copy from
    // pageable memory
    soap_status st = stage_to_device(c, flux, in_bytes, c->ws_specin.ptr);
    if (st != SOAP_OK) return st;
    dflux = c->ws_specin.ptr;
  }
  const int nlb = soap::ccf_line_blocks(nl);
  const size_t ccf_elems = (size_t)n_spec * c->mask_nv;
  HIP_TRY(grow(c->ws_ccf, c->esize * ccf_elems * nlb));
  double* dccf = (ccf_out && ccf_on_device) ? ccf_out : nullptr;
  if (!dccf) {
    HIP_TRY(grow(c->ws_ccfout, sizeof(double) * ccf_elems));
    dccf = static_cast<double*>(c->ws_ccfout.ptr);
  }
  {
    StageTimer t(c, ST_CCF);
    HIP_TRY(soap::launch_ccf(c, dflux, n_spec, nl, c->ws_ccf.ptr));
    t.done();
  }
  c->ccf_calls++;
  soap_rv* drv = nullptr;
  if (rv_out) {
    drv = rv_on_device ? rv_out : nullptr;
    if (!drv) {
      HIP_TRY(grow(c->ws_rv, sizeof(soap_rv) * (size_t)n_spec));
      drv = static_cast<soap_rv*>(c->ws_rv.ptr);
    }
  }
  {
    StageTimer t(c, ST_GFIT);
    HIP_TRY(soap::launch_ccf_fit(c, nl, c->ws_ccf.ptr, n_spec, dccf, drv));
    t.done();
  }
  // host outputs: blocking copies once the stream is idle
  const bool rv_host = rv_out && !rv_on_device, ccf_host = ccf_out && !ccf_on_device;
  if (rv_host || ccf_host || !flux_on_device) HIP_TRY(hipStreamSynchronize(c->stream));
  if (rv_host) HIP_TRY(hipMemcpy(rv_out, drv, sizeof(soap_rv) * n_spec, hipMemcpyDeviceToHost));
  if (ccf_host) HIP_TRY(hipMemcpy(ccf_out, dccf, sizeof(double) * ccf_elems, hipMemcpyDeviceToHost));
  return SOAP_OK;
}

SOAP_API soap_status soap_ccf_linear_rv(soap_ctx* c, const float* coef, int64_t n, int32_t k, const double* base,
                                        const double* basis, double* ccf_out, soap_rv* rv_out) {
  if (!c) return SOAP_ERR_ARG;
  std::string& err = c->err;
  ARG_CHECK(coef && base && basis, "coef, base and basis must be device arrays");
  ARG_CHECK(n >= 1 && n <= (int64_t(1) << 24), "n must be in [1, 2^24]");
  ARG_CHECK(k >= 1 && k <= 4096, "k must be in [1, 4096]");
  if (!c->mask_valid) {
    setf(c->err, "no mask yet: call soap_ccf_rv with the mask first");
    return SOAP_ERR_STATE;
  }
  double* lin = ccf_out;
  if (!lin) {
    HIP_TRY(grow(c->ws_ccfout, sizeof(double) * (size_t)n * c->mask_nv));
    lin = static_cast<double*>(c->ws_ccfout.ptr);
  }
  // the fit reads each row into registers before writing it back, so the
  // linear CCF and the output may share storage
  HIP_TRY(soap::launch_ccf_linear_fit(c, coef, n, k, base, basis, lin, lin, rv_out));
  return SOAP_OK;
}

SOAP_API soap_status soap_surrogate_rv(soap_ctx* c, const float* coef, const float* members, int64_t n,
                                       int32_t n_ens, int32_t k, const double* base, const int32_t* base_index,
                                       int32_t n_base, const double* basis, double calib, double threshold_kms,
                                       soap_rv* rv_out, double* rv_kms, double* err_kms, int32_t* fallback) {
  if (!c) return SOAP_ERR_ARG;
  std::string& err = c->err;
  ARG_CHECK(coef && members && base && basis && rv_kms && fallback, "a required device array is NULL");
  ARG_CHECK(n >= 1 && n <= (int64_t(1) << 24), "n must be in [1, 2^24]");
  ARG_CHECK(k >= 1 && k <= 4096, "k must be in [1, 4096]");
  ARG_CHECK(n_ens >= 2 && n_ens <= 16, "n_ens must be in [2, 16]");
  ARG_CHECK(is_finite(calib) && calib >= 0.0 && !std::isnan(threshold_kms), "calib or threshold invalid");
  if (!c->mask_valid) {
    setf(c->err, "no mask yet: call soap_ccf_rv with the mask first");
    return SOAP_ERR_STATE;
  }
  ARG_CHECK(!base_index || n_base >= 1, "n_base must be >= 1 with base_index");
  const size_t wb = soap::sg_rv_work_bytes(c, n);
  if (c->ws_sg.bytes < wb) {
    // the workspace is replaced only with the stream idle
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(grow(c->ws_sg, wb));
  }
  HIP_TRY(soap::launch_sg_rv(c, coef, members, n, n_ens, k, base, base_index, n_base, basis, calib, threshold_kms,
                             rv_out, rv_kms, err_kms, fallback, c->ws_sg.ptr));
  return SOAP_OK;
}

SOAP_API soap_status soap_profile_enable(soap_ctx* c, int32_t on) {
  if (!c) return SOAP_ERR_ARG;
  HIP_TRY(hipStreamSynchronize(c->side));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  c->pending.clear();
  for (double& v : c->stage_ms) v = 0.0;
  c->active_calls = c->ccf_calls = 0;
  c->prof = on != 0;
  return SOAP_OK;
}

SOAP_API soap_status soap_profile_read(soap_ctx* c, soap_profile* out) {
  if (!c) return SOAP_ERR_ARG;
  std::string& err = c->err;
  ARG_CHECK(out != nullptr, "out is NULL");
  HIP_TRY(hipStreamSynchronize(c->side));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (auto& p : c->pending) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, p.a, p.b);
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
    if (e == hipSuccess) c->stage_ms[p.stage] += ms;
  }
  c->pending.clear();
  out->weights_ms = c->stage_ms[ST_WEIGHTS];
  out->compact_ms = c->stage_ms[ST_COMPACT];
  out->apply_ms = c->stage_ms[ST_APPLY];
  out->ccf_ms = c->stage_ms[ST_CCF];
  out->gfit_ms = c->stage_ms[ST_GFIT];
  out->lsf_ms = c->stage_ms[ST_LSF];
  out->active_calls = c->active_calls;
  out->ccf_calls = c->ccf_calls;
  out->src_arrays = out->con_arrays = 0;
  out->taps_nonzero = out->taps_offsets = out->fma_issued = 0;
  out->last_phases = c->last_phases;
  if (c->last_phases > 0) {
    // distinct inputs the last apply walked, from its virtual-group lists
    const int n_chunks = (c->last_phases + c->last_pc - 1) / c->last_pc;
    const size_t wb = (size_t)soap::win_bytes(c->last_pc, (int)c->esize);
    std::vector<int> nvg(n_chunks);
    std::vector<unsigned char> vg((size_t)n_chunks * c->last_vg_cap * wb);
    const soap_ctx::PrepSet& S = c->prep[c->last_prep];
    HIP_TRY(hipMemcpy(nvg.data(), S.nvg.ptr, sizeof(int) * n_chunks, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(vg.data(), S.vg.ptr, vg.size(), hipMemcpyDeviceToHost));
    std::vector<char> src(3 * c->B, 0), con(3 * c->B, 0);
    const bool per_pixel = c->cmode != SOAP_CONTRAST_SCALAR;
    const bool spot_rows = c->con_spot_stride != 0;  // one spot contrast row per bin
    for (int ch = 0; ch < n_chunks; ++ch)
      for (int v = 0; v < nvg[ch]; ++v) {
        soap::WinHead h;
        const unsigned char* rec = vg.data() + ((size_t)ch * c->last_vg_cap + v) * wb;
        std::memcpy(&h, rec, sizeof(h));
        {
          // taps[q][p] after the header, float or double per the precision;
          // one mask bit per (offset, pair of phases) with a non-zero tap:
          // each bit costs two FMAs per pixel, each offset with a bit one
          // difference formation
          int pairs = 0, offs = 0;
          for (unsigned m = h.gmask; m; m &= m - 1) ++pairs;
          for (int q = 0; q < soap::APPLY_JW; ++q)
            if ((h.gmask >> (q * (c->last_pc / 2))) & ((1u << (c->last_pc / 2)) - 1u)) ++offs;
          out->fma_issued += (int64_t)pairs * 2 + offs;
          for (int q = 0; q < soap::APPLY_JW; ++q) {
            bool any = false;
            for (int pp = 0; pp < c->last_pc; ++pp) {
              double tap;
              if (c->prec == SOAP_PREC_FP32) {
                float f;
                std::memcpy(&f, rec + 16 + sizeof(float) * ((size_t)q * c->last_pc + pp), sizeof f);
                tap = f;
              } else {
                std::memcpy(&tap, rec + 16 + sizeof(double) * ((size_t)q * c->last_pc + pp), sizeof tap);
              }
              if (tap != 0.0) {
                ++out->taps_nonzero;
                any = true;
              }
            }
            if (any) ++out->taps_offsets;
          }
        }
        const int t = h.t, b = h.b;
        if (t == 0) {
          src[b] = 1;
          continue;
        }
        if (c->last_paired) src[b] = 1;  // the implied quiet removal
        if (c->last_effect == SOAP_EFFECT_FLUX) src[b] = 1;
        else src[t * c->B + b] = 1;
        // spot contrast is one array for every bin, facula one per bin
        if (per_pixel && c->last_effect != SOAP_EFFECT_BCONV)
          con[(t == SOAP_SPOT && !spot_rows) ? SOAP_SPOT * c->B : t * c->B + b] = 1;
      }
    for (char x : src) out->src_arrays += x;
    for (char x : con) out->con_arrays += x;
  }
  return SOAP_OK;
}

SOAP_API soap_status soap_sync(soap_ctx* c) {
  if (!c) return SOAP_ERR_ARG;
  HIP_TRY(hipStreamSynchronize(c->side));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return SOAP_OK;
}

SOAP_API void soap_destroy(soap_ctx* c) { destroy_ctx(c); }
