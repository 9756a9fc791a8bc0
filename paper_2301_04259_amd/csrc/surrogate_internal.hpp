// Internal declarations of the surrogate network (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "soap.h"

namespace soap {

constexpr int SG_K0 = 32;            // input width padded to one MFMA K step
constexpr int SG_RAW = 8;            // raw sample description (soap_surrogate_features)
constexpr int SG_FEATURES = 12;      // network inputs made from it
constexpr int SG_COLSUM_ROWS = 128;  // rows per partial column sum

enum { MM_PLAIN = 0, MM_HIDDEN = 1, MM_OUTPUT = 2, MM_DHIDDEN = 3 };

// offsets (elements) of one member's parameters on the device: W1 [SG_K0][H]
// (rows >= n_in zero), b1 [H], W2 [H][H], b2 [H], W3 [H][O], b3 [O]
struct SgLayout {
  int64_t W1, b1, W2, b2, W3, b3, n_params;
};

}  // namespace soap

struct soap_surrogate {
  int n_in = 0, hidden = 0, n_out = 0, n_ens = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  soap::SgLayout lay{};
  int64_t step = 0;
  std::string err;
  // parameters and optimiser state, [n_ens][lay.n_params]
  float* P = nullptr;
  float* G = nullptr;
  float* M = nullptr;
  float* V = nullptr;
  __bf16* Pb = nullptr;
  // per-batch activations (grown on demand)
  int cap = 0;  // rows the buffers hold
  __bf16* X = nullptr;                // [cap][SG_K0]
  float *Z1 = nullptr, *Z2 = nullptr;  // [E][cap][H]
  __bf16 *H1 = nullptr, *H2 = nullptr;
  float* Y = nullptr;                 // [E][cap][O]
  __bf16* dY = nullptr;
  float* dYf = nullptr;
  float *dZf = nullptr, *dZf2 = nullptr;  // [E][cap][H]
  __bf16 *dZb = nullptr, *dZb2 = nullptr;
  float* row_se = nullptr;  // [E][cap]
  float* colpart = nullptr; // [E][cap / SG_COLSUM_ROWS][max(H, O)] partial column sums
  float* loss = nullptr;    // [E]
};

namespace soap {
hipError_t sg_forward(soap_surrogate* s, const float* x, int B);
hipError_t sg_backward(soap_surrogate* s, const float* target, int B);
hipError_t sg_adam(soap_surrogate* s, float lr);
hipError_t sg_sync_bf16(soap_surrogate* s);
hipError_t sg_ens_mean(soap_surrogate* s, int B, float* mean);
hipError_t sg_gate(hipStream_t st, const soap_rv* rv, int64_t n, int E, double calib, double thr, double* rv_kms,
                   double* err_kms, int* fallback);
// network inputs [n][SG_FEATURES] of raw sample descriptions [n][SG_RAW]
hipError_t sg_features(hipStream_t st, int64_t n, const double* raw, float* x);
hipError_t sg_pca_project(hipStream_t st, int n, int P, int k, const float* D, int64_t ldd, const float* mean,
                          const int* mean_idx, int n_mean, const float* V, float* coef);
}  // namespace soap
