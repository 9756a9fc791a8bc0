// C ABI of the surrogate network and of the PCA projection (include/soap.h).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "devmem.hpp"
#include "surrogate_internal.hpp"

#define SOAP_API extern "C" __attribute__((visibility("default")))

namespace {

void sg_setf(std::string& err, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  err = buf;
}

#define SG_ARG(cond, ...)               \
  do {                                  \
    if (!(cond)) {                      \
      sg_setf(s->err, __VA_ARGS__);     \
      return SOAP_ERR_ARG;              \
    }                                   \
  } while (0)

#define SG_HIP(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                        \
      sg_setf(s->err, "%s failed: %s%s", #x, hipGetErrorString(e_),              \
              e_ == hipErrorOutOfMemory ? soap::dev_cap_note() : "");              \
      return e_ == hipErrorOutOfMemory ? SOAP_ERR_OOM : SOAP_ERR_HIP;              \
    }                                                                              \
  } while (0)

// counter-based generator (SplitMix64) for the initial weights
uint64_t splitmix(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double unit(uint64_t& x) { return (double)(splitmix(x) >> 11) * (1.0 / 9007199254740992.0); }

// natural layout offsets (what callers see): W1 [n_in][H], b1, W2, b2, W3, b3
struct Natural {
  int64_t W1, b1, W2, b2, W3, b3, n;
};

Natural natural(const soap_surrogate* s) {
  Natural a;
  const int64_t H = s->hidden, O = s->n_out;
  a.W1 = 0;
  a.b1 = a.W1 + (int64_t)s->n_in * H;
  a.W2 = a.b1 + H;
  a.b2 = a.W2 + H * H;
  a.W3 = a.b2 + H;
  a.b3 = a.W3 + H * O;
  a.n = a.b3 + O;
  return a;
}

// copy one member between the natural (host) and the padded (device) layout
void to_device_layout(const soap_surrogate* s, const float* nat, std::vector<float>& dev) {
  const Natural a = natural(s);
  const soap::SgLayout& L = s->lay;
  const int64_t H = s->hidden, O = s->n_out;
  dev.assign(L.n_params, 0.f);
  for (int k = 0; k < s->n_in; ++k)
    std::memcpy(&dev[L.W1 + k * H], nat + a.W1 + k * H, sizeof(float) * H);
  std::memcpy(&dev[L.b1], nat + a.b1, sizeof(float) * H);
  std::memcpy(&dev[L.W2], nat + a.W2, sizeof(float) * H * H);
  std::memcpy(&dev[L.b2], nat + a.b2, sizeof(float) * H);
  std::memcpy(&dev[L.W3], nat + a.W3, sizeof(float) * H * O);
  std::memcpy(&dev[L.b3], nat + a.b3, sizeof(float) * O);
}

void to_natural_layout(const soap_surrogate* s, const std::vector<float>& dev, float* nat) {
  const Natural a = natural(s);
  const soap::SgLayout& L = s->lay;
  const int64_t H = s->hidden, O = s->n_out;
  for (int k = 0; k < s->n_in; ++k)
    std::memcpy(nat + a.W1 + k * H, &dev[L.W1 + k * H], sizeof(float) * H);
  std::memcpy(nat + a.b1, &dev[L.b1], sizeof(float) * H);
  std::memcpy(nat + a.W2, &dev[L.W2], sizeof(float) * H * H);
  std::memcpy(nat + a.b2, &dev[L.b2], sizeof(float) * H);
  std::memcpy(nat + a.W3, &dev[L.W3], sizeof(float) * H * O);
  std::memcpy(nat + a.b3, &dev[L.b3], sizeof(float) * O);
}

template <typename T>
hipError_t alloc(T*& p, size_t n) {
  if (p) (void)soap::dev_free(p);
  p = nullptr;
  return soap::dev_malloc((void**)&p, sizeof(T) * std::max<size_t>(n, 1));
}

void free_all(soap_surrogate* s) {
  void* ps[] = {s->P, s->G, s->M, s->V, s->Pb, s->X, s->Z1, s->Z2, s->H1, s->H2, s->Y, s->dY, s->dYf,
                s->dZf, s->dZf2, s->dZb, s->dZb2, s->row_se, s->loss, s->colpart};
  for (void* p : ps)
    if (p) (void)soap::dev_free(p);
}

soap_status ensure_batch(soap_surrogate* s, int B) {
  if (B <= s->cap) return SOAP_OK;
  SG_HIP(hipStreamSynchronize(s->stream));
  const size_t E = s->n_ens, H = s->hidden, O = s->n_out;
  SG_HIP(alloc(s->X, (size_t)B * soap::SG_K0));
  SG_HIP(alloc(s->Z1, E * B * H));
  SG_HIP(alloc(s->Z2, E * B * H));
  SG_HIP(alloc(s->H1, E * B * H));
  SG_HIP(alloc(s->H2, E * B * H));
  SG_HIP(alloc(s->Y, E * B * O));
  SG_HIP(alloc(s->dY, E * B * O));
  SG_HIP(alloc(s->dYf, E * B * O));
  SG_HIP(alloc(s->dZf, E * B * H));
  SG_HIP(alloc(s->dZf2, E * B * H));
  SG_HIP(alloc(s->dZb, E * B * H));
  SG_HIP(alloc(s->dZb2, E * B * H));
  SG_HIP(alloc(s->row_se, E * B));
  SG_HIP(alloc(s->colpart, E * (((size_t)B + soap::SG_COLSUM_ROWS - 1) / soap::SG_COLSUM_ROWS) * std::max(H, O)));
  s->cap = B;
  return SOAP_OK;
}

constexpr uint32_t SG_MAGIC = 0x53475231u;  // file tag

}  // namespace

SOAP_API soap_status soap_surrogate_create(int32_t n_in, int32_t hidden, int32_t n_out, int32_t n_ensemble,
                                           uint64_t seed, void* hip_stream, soap_surrogate** out) {
  if (!out) return SOAP_ERR_ARG;
  *out = nullptr;
  if (n_in < 1 || n_in > soap::SG_K0 || hidden < 32 || hidden > 4096 || hidden % 32 != 0 || n_out < 32 ||
      n_out > 4096 || n_out % 32 != 0 || n_ensemble < 1 || n_ensemble > 16)
    return SOAP_ERR_ARG;
  soap_surrogate* s = new soap_surrogate;
  s->n_in = n_in;
  s->hidden = hidden;
  s->n_out = n_out;
  s->n_ens = n_ensemble;
  s->stream = static_cast<hipStream_t>(hip_stream);
  const int64_t H = hidden, O = n_out;
  soap::SgLayout& L = s->lay;
  L.W1 = 0;
  L.b1 = L.W1 + (int64_t)soap::SG_K0 * H;
  L.W2 = L.b1 + H;
  L.b2 = L.W2 + H * H;
  L.W3 = L.b2 + H;
  L.b3 = L.W3 + H * O;
  L.n_params = L.b3 + O;
  auto fail = [&](soap_status st) {
    free_all(s);
    delete s;
    return st;
  };
  if (hipGetDevice(&s->device) != hipSuccess) return fail(SOAP_ERR_HIP);
  const size_t np = (size_t)n_ensemble * L.n_params;
  if (alloc(s->P, np) != hipSuccess || alloc(s->G, np) != hipSuccess || alloc(s->M, np) != hipSuccess ||
      alloc(s->V, np) != hipSuccess || alloc(s->Pb, np) != hipSuccess || alloc(s->loss, n_ensemble) != hipSuccess)
    return fail(SOAP_ERR_OOM);
  // Glorot-uniform weights from the seeded generator (one stream per
  // member), zero biases
  std::vector<float> host(np, 0.f);
  for (int e = 0; e < n_ensemble; ++e) {
    uint64_t st = seed * 0x100000001B3ull + (uint64_t)e * 0x9E3779B97F4A7C15ull + 1;
    float* p = host.data() + (size_t)e * L.n_params;
    auto fill = [&](int64_t off, int64_t rows, int64_t cols, int64_t fan_in, int64_t fan_out) {
      const double a = std::sqrt(6.0 / (double)(fan_in + fan_out));
      for (int64_t r = 0; r < rows; ++r)
        for (int64_t c = 0; c < cols; ++c) p[off + r * cols + c] = (float)((2.0 * unit(st) - 1.0) * a);
    };
    fill(L.W1, n_in, H, n_in, H);
    fill(L.W2, H, H, H, H);
    fill(L.W3, H, O, H, O);
  }
  if (hipMemcpy(s->P, host.data(), sizeof(float) * np, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(s->G, 0, sizeof(float) * np) != hipSuccess || hipMemset(s->M, 0, sizeof(float) * np) != hipSuccess ||
      hipMemset(s->V, 0, sizeof(float) * np) != hipSuccess || soap::sg_sync_bf16(s) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess)
    return fail(SOAP_ERR_HIP);
  *out = s;
  return SOAP_OK;
}

SOAP_API int64_t soap_surrogate_n_params(const soap_surrogate* s) { return s ? natural(s).n : -1; }

SOAP_API soap_status soap_surrogate_train_step(soap_surrogate* s, const float* x_dev, const float* y_dev,
                                               int32_t batch, float lr, float* loss_out) {
  if (!s) return SOAP_ERR_ARG;
  SG_ARG(x_dev && y_dev, "x and y must be device arrays");
  SG_ARG(batch >= 32 && batch % 32 == 0 && batch <= (1 << 20), "batch must be a multiple of 32 in [32, 2^20]");
  SG_ARG(std::isfinite(lr) && lr > 0.f, "lr must be > 0");
  soap_status st = ensure_batch(s, batch);
  if (st != SOAP_OK) return st;
  SG_HIP(soap::sg_forward(s, x_dev, batch));
  SG_HIP(soap::sg_backward(s, y_dev, batch));
  SG_HIP(soap::sg_adam(s, lr));
  if (loss_out) {
    std::vector<float> l(s->n_ens);
    SG_HIP(hipStreamSynchronize(s->stream));
    SG_HIP(hipMemcpy(l.data(), s->loss, sizeof(float) * s->n_ens, hipMemcpyDeviceToHost));
    double a = 0.0;
    for (float v : l) a += v;
    *loss_out = (float)(a / s->n_ens);
  }
  return SOAP_OK;
}

SOAP_API soap_status soap_surrogate_predict(soap_surrogate* s, const float* x_dev, int32_t batch, float* coef_dev,
                                            float* members_dev) {
  if (!s) return SOAP_ERR_ARG;
  SG_ARG(x_dev && coef_dev, "x and coef must be device arrays");
  SG_ARG(batch >= 16 && batch % 16 == 0 && batch <= (1 << 20), "batch must be a multiple of 16 in [16, 2^20]");
  soap_status st = ensure_batch(s, batch);
  if (st != SOAP_OK) return st;
  SG_HIP(soap::sg_forward(s, x_dev, batch));
  SG_HIP(soap::sg_ens_mean(s, batch, coef_dev));
  if (members_dev)
    SG_HIP(hipMemcpyAsync(members_dev, s->Y, sizeof(float) * (size_t)s->n_ens * batch * s->n_out,
                          hipMemcpyDeviceToDevice, s->stream));
  return SOAP_OK;
}

SOAP_API soap_status soap_surrogate_get_params(const soap_surrogate* s_, int32_t member, float* out) {
  soap_surrogate* s = const_cast<soap_surrogate*>(s_);
  if (!s) return SOAP_ERR_ARG;
  SG_ARG(out && member >= 0 && member < s->n_ens, "bad member or NULL output");
  std::vector<float> dev(s->lay.n_params);
  SG_HIP(hipStreamSynchronize(s->stream));
  SG_HIP(hipMemcpy(dev.data(), s->P + (size_t)member * s->lay.n_params, sizeof(float) * dev.size(),
                   hipMemcpyDeviceToHost));
  to_natural_layout(s, dev, out);
  return SOAP_OK;
}

SOAP_API soap_status soap_surrogate_get_grads(const soap_surrogate* s_, int32_t member, float* out) {
  soap_surrogate* s = const_cast<soap_surrogate*>(s_);
  if (!s) return SOAP_ERR_ARG;
  SG_ARG(out && member >= 0 && member < s->n_ens, "bad member or NULL output");
  std::vector<float> dev(s->lay.n_params);
  SG_HIP(hipStreamSynchronize(s->stream));
  SG_HIP(hipMemcpy(dev.data(), s->G + (size_t)member * s->lay.n_params, sizeof(float) * dev.size(),
                   hipMemcpyDeviceToHost));
  to_natural_layout(s, dev, out);
  return SOAP_OK;
}

SOAP_API soap_status soap_surrogate_set_params(soap_surrogate* s, int32_t member, const float* in) {
  if (!s) return SOAP_ERR_ARG;
  SG_ARG(in && member >= 0 && member < s->n_ens, "bad member or NULL input");
  std::vector<float> dev;
  to_device_layout(s, in, dev);
  SG_HIP(hipStreamSynchronize(s->stream));
  SG_HIP(hipMemcpy(s->P + (size_t)member * s->lay.n_params, dev.data(), sizeof(float) * dev.size(),
                   hipMemcpyHostToDevice));
  SG_HIP(soap::sg_sync_bf16(s));
  SG_HIP(hipStreamSynchronize(s->stream));
  return SOAP_OK;
}

SOAP_API soap_status soap_surrogate_save(const soap_surrogate* s_, const char* path) {
  soap_surrogate* s = const_cast<soap_surrogate*>(s_);
  if (!s) return SOAP_ERR_ARG;
  SG_ARG(path != nullptr, "path is NULL");
  const size_t np = (size_t)s->n_ens * s->lay.n_params;
  std::vector<float> p(np), m(np), v(np);
  SG_HIP(hipStreamSynchronize(s->stream));
  SG_HIP(hipMemcpy(p.data(), s->P, sizeof(float) * np, hipMemcpyDeviceToHost));
  SG_HIP(hipMemcpy(m.data(), s->M, sizeof(float) * np, hipMemcpyDeviceToHost));
  SG_HIP(hipMemcpy(v.data(), s->V, sizeof(float) * np, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  if (!f) {
    sg_setf(s->err, "cannot open %s for writing", path);
    return SOAP_ERR_ARG;
  }
  const int32_t hdr[6] = {(int32_t)SG_MAGIC, s->n_in, s->hidden, s->n_out, s->n_ens, 0};
  const int64_t step = s->step;
  bool ok = std::fwrite(hdr, sizeof hdr, 1, f) == 1 && std::fwrite(&step, sizeof step, 1, f) == 1 &&
            std::fwrite(p.data(), sizeof(float), np, f) == np && std::fwrite(m.data(), sizeof(float), np, f) == np &&
            std::fwrite(v.data(), sizeof(float), np, f) == np;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) {
    sg_setf(s->err, "short write to %s", path);
    return SOAP_ERR_ARG;
  }
  return SOAP_OK;
}

SOAP_API soap_status soap_surrogate_load(soap_surrogate* s, const char* path) {
  if (!s) return SOAP_ERR_ARG;
  SG_ARG(path != nullptr, "path is NULL");
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    sg_setf(s->err, "cannot open %s", path);
    return SOAP_ERR_ARG;
  }
  int32_t hdr[6];
  int64_t step = 0;
  const size_t np = (size_t)s->n_ens * s->lay.n_params;
  std::vector<float> p(np), m(np), v(np);
  bool ok = std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == (int32_t)SG_MAGIC && hdr[1] == s->n_in &&
            hdr[2] == s->hidden && hdr[3] == s->n_out && hdr[4] == s->n_ens &&
            std::fread(&step, sizeof step, 1, f) == 1 && std::fread(p.data(), sizeof(float), np, f) == np &&
            std::fread(m.data(), sizeof(float), np, f) == np && std::fread(v.data(), sizeof(float), np, f) == np;
  std::fclose(f);
  if (!ok) {
    sg_setf(s->err, "%s is not a surrogate file of this shape", path);
    return SOAP_ERR_ARG;
  }
  SG_HIP(hipStreamSynchronize(s->stream));
  SG_HIP(hipMemcpy(s->P, p.data(), sizeof(float) * np, hipMemcpyHostToDevice));
  SG_HIP(hipMemcpy(s->M, m.data(), sizeof(float) * np, hipMemcpyHostToDevice));
  SG_HIP(hipMemcpy(s->V, v.data(), sizeof(float) * np, hipMemcpyHostToDevice));
  s->step = step;
  SG_HIP(soap::sg_sync_bf16(s));
  SG_HIP(hipStreamSynchronize(s->stream));
  return SOAP_OK;
}

SOAP_API const char* soap_surrogate_last_error(const soap_surrogate* s) { return s ? s->err.c_str() : "NULL"; }

SOAP_API void soap_surrogate_destroy(soap_surrogate* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  free_all(s);
  delete s;
}

SOAP_API soap_status soap_pca_project(const float* d_dev, int64_t n, int64_t n_pix, int64_t ld, const float* mean_dev,
                                      const int32_t* mean_index, int32_t n_mean, const float* basis_dev, int32_t k,
                                      float* coef_dev, void* hip_stream) {
  if (!d_dev || !mean_dev || !basis_dev || !coef_dev) return SOAP_ERR_ARG;
  if (n < 1 || n > (int64_t(1) << 31) / 64 || n_pix < 1 || n_pix > (int64_t(1) << 30) || ld < n_pix || k < 1 ||
      k > 4096)
    return SOAP_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (mean_index && n_mean < 1) return SOAP_ERR_ARG;
  if (soap::sg_pca_project(st, (int)n, (int)n_pix, k, d_dev, ld, mean_dev, mean_index, n_mean, basis_dev,
                           coef_dev) != hipSuccess)
    return SOAP_ERR_HIP;
  return SOAP_OK;
}

SOAP_API soap_status soap_surrogate_features(const double* raw_dev, int64_t n, float* x_dev, void* hip_stream) {
  if (!raw_dev || !x_dev || n < 1 || n > (int64_t(1) << 26)) return SOAP_ERR_ARG;
  if (soap::sg_features(static_cast<hipStream_t>(hip_stream), n, raw_dev, x_dev) != hipSuccess) return SOAP_ERR_HIP;
  return SOAP_OK;
}

SOAP_API soap_status soap_surrogate_gate(const soap_rv* rv, int64_t n, int32_t n_ens, double calib,
                                         double threshold_kms, double* rv_kms, double* err_kms, int32_t* fallback,
                                         void* hip_stream) {
  if (!rv || !rv_kms || !fallback || n < 1 || n > (int64_t(1) << 24) || n_ens < 2 || n_ens > 16 ||
      !std::isfinite(calib) || calib < 0.0 || std::isnan(threshold_kms))
    return SOAP_ERR_ARG;
  if (soap::sg_gate(static_cast<hipStream_t>(hip_stream), rv, n, n_ens, calib, threshold_kms, rv_kms, err_kms,
                    fallback) != hipSuccess)
    return SOAP_ERR_HIP;
  return SOAP_OK;
}
