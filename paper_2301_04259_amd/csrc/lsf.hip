// Resolution lowering to the instrument's line-spread function (the last step
// of Algorithms 2 and 5: each final spectrum is lowered to the resolution of
// the spectrograph).
//
// The line-spread function is a Gaussian of full width at half maximum
// lambda / R, which on the log-uniform grid is the same width at every pixel,
// sigma = 1 / (R dln 2 sqrt(2 ln 2)) pixels.  The kernel is that Gaussian
// sampled at whole-pixel offsets |k| <= K = ceil(4 sigma), normalised to sum
// 1 (on the host, in double), and out[m] = sum_k w_k F[clamp(m - k)] with the
// end values held, k in increasing order.
//
// One block of 256 threads per (spectrum, tile of 1024 pixels): the tile and
// its K-pixel halos are staged in LDS with coalesced loads (16-byte loads for
// the tile body where the row allows), then each thread forms 4 consecutive
// outputs from 4 + 2 KP staged samples held in registers (KP >= K, the taps
// past K are zero) and writes them with one 16-byte store where aligned.  The
// kernel reads each input sample once plus the halos and writes each output
// once: HBM-bound, 2 x n_spec x n_pix x sizeof(T) bytes.
#include <cmath>

#include "soap_internal.hpp"

namespace soap {

namespace {

constexpr int LSF_THREADS = 256;
constexpr int LSF_TILE = 4 * LSF_THREADS;

template <typename T>
struct LsfTaps {
  T w[2 * LSF_KMAX + 1];  // w[KP + k] for k = -KP .. KP (zero past K)
};

template <typename T, int KP>
__global__ void __launch_bounds__(LSF_THREADS) k_lsf(int64_t P, int64_t tiles, int K, int vec_in, int vec_out,
                                                     LsfTaps<T> taps, const T* __restrict__ in,
                                                     T* __restrict__ out) {
  __shared__ __align__(16) T s[LSF_TILE + 2 * KP + 4];
  const int64_t b = blockIdx.x;
  const int64_t row = b / tiles;
  const int64_t m0 = (b - row * tiles) * LSF_TILE;
  const T* src = in + row * P;
  T* dst = out + row * P;
  const int t = threadIdx.x;
  // s[KP + i] holds F[clamp(m0 + i)] for i in [-KP, LSF_TILE + KP)
  {
    const int64_t m = m0 + 4 * t;
    if (vec_in && m + 4 <= P) {
      if constexpr (sizeof(T) == 4) {
        const float4 v = *reinterpret_cast<const float4*>(src + m);
        s[KP + 4 * t + 0] = v.x;
        s[KP + 4 * t + 1] = v.y;
        s[KP + 4 * t + 2] = v.z;
        s[KP + 4 * t + 3] = v.w;
      } else {
        const double2 u = reinterpret_cast<const double2*>(src + m)[0];
        const double2 v = reinterpret_cast<const double2*>(src + m)[1];
        s[KP + 4 * t + 0] = u.x;
        s[KP + 4 * t + 1] = u.y;
        s[KP + 4 * t + 2] = v.x;
        s[KP + 4 * t + 3] = v.y;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t q = m + r;
        s[KP + 4 * t + r] = src[q < P ? q : P - 1];
      }
    }
  }
  if (t < 2 * KP) {
    // halos: KP samples before the tile, KP after
    const int i = t < KP ? t - KP : LSF_TILE + (t - KP);
    int64_t q = m0 + i;
    q = q < 0 ? 0 : (q >= P ? P - 1 : q);
    s[KP + i] = src[q];
  }
  __syncthreads();
  // x[j] = s[4t + j] = F[clamp(m0 + 4t + j - KP)], j < 4 + 2 KP
  T x[4 + 2 * KP];
#pragma unroll
  for (int j = 0; j < 4 + 2 * KP; j += 4) {
    if constexpr (sizeof(T) == 4) {
      const float4 v = *reinterpret_cast<const float4*>(&s[4 * t + j]);
      x[j] = v.x;
      x[j + 1] = v.y;
      x[j + 2] = v.z;
      x[j + 3] = v.w;
    } else {
      const double2 u = *reinterpret_cast<const double2*>(&s[4 * t + j]);
      const double2 v = *reinterpret_cast<const double2*>(&s[4 * t + j + 2]);
      x[j] = u.x;
      x[j + 1] = u.y;
      x[j + 2] = v.x;
      x[j + 3] = v.y;
    }
  }
  // out[m0 + 4t + r] = sum_k w_k F[m0 + 4t + r - k] = sum_k w_k x[r - k + KP]
  T acc[4] = {T(0), T(0), T(0), T(0)};
  const int kb = KP - K;  // first non-zero tap (k = -K)
#pragma unroll
  for (int kk = 0; kk <= 2 * KP; ++kk) {
    if (kk < kb || kk > 2 * KP - kb) continue;  // uniform: zero taps past K
    const T w = taps.w[kk];
    const int k = kk - KP;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = fma(w, x[r - k + KP], acc[r]);
  }
  const int64_t m = m0 + 4 * t;
  if (vec_out && m + 4 <= P) {
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<float4*>(dst + m) = make_float4(acc[0], acc[1], acc[2], acc[3]);
    } else {
      reinterpret_cast<double2*>(dst + m)[0] = make_double2(acc[0], acc[1]);
      reinterpret_cast<double2*>(dst + m)[1] = make_double2(acc[2], acc[3]);
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (m + r < P) dst[m + r] = acc[r];
  }
}

template <typename T, int KP>
hipError_t launch_kp(const LsfPlan& pl, int64_t P, int64_t n_spec, const void* in, void* out, hipStream_t st) {
  LsfTaps<T> taps;
  for (int i = 0; i < 2 * LSF_KMAX + 1; ++i) taps.w[i] = T(0);
  for (int k = -pl.K; k <= pl.K; ++k) taps.w[KP + k] = (T)pl.w[k + pl.K];
  const int64_t tiles = (P + LSF_TILE - 1) / LSF_TILE;
  const size_t al = 4 * sizeof(T);
  const int vec_in = (P % 4 == 0) && (reinterpret_cast<uintptr_t>(in) % al == 0);
  const int vec_out = (P % 4 == 0) && (reinterpret_cast<uintptr_t>(out) % al == 0);
  hipLaunchKernelGGL((k_lsf<T, KP>), dim3((unsigned)(tiles * n_spec)), dim3(LSF_THREADS), 0, st, P, tiles, pl.K,
                     vec_in, vec_out, taps, static_cast<const T*>(in), static_cast<T*>(out));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_t(const LsfPlan& pl, int64_t P, int64_t n_spec, const void* in, void* out, hipStream_t st) {
  if (pl.K <= 4) return launch_kp<T, 4>(pl, P, n_spec, in, out, st);
  if (pl.K <= 8) return launch_kp<T, 8>(pl, P, n_spec, in, out, st);
  if (pl.K <= 16) return launch_kp<T, 16>(pl, P, n_spec, in, out, st);
  static_assert(LSF_KMAX == 32, "widest template instance");
  return launch_kp<T, 32>(pl, P, n_spec, in, out, st);
}

}  // namespace

bool lsf_plan(double resolution, double dln, LsfPlan* pl) {
  const double sigma = 1.0 / (resolution * dln * 2.0 * std::sqrt(2.0 * std::log(2.0)));
  const double kf = std::ceil(4.0 * sigma);
  if (!(kf >= 0.0) || kf > LSF_KMAX) return false;
  pl->K = (int)kf;
  double sum = 0.0;
  for (int k = -pl->K; k <= pl->K; ++k) {
    const double z = k / sigma;
    pl->w[k + pl->K] = std::exp(-0.5 * z * z);
    sum += pl->w[k + pl->K];
  }
  for (int k = -pl->K; k <= pl->K; ++k) pl->w[k + pl->K] /= sum;
  pl->sigma = sigma;
  return true;
}

int64_t lsf_max_spectra(int64_t P) {
  const int64_t tiles = (P + LSF_TILE - 1) / LSF_TILE;
  return ((int64_t(1) << 31) - 1) / tiles;
}

hipError_t launch_lsf(soap_ctx* c, const LsfPlan& pl, const void* in, void* out, int64_t n_spec, hipStream_t st) {
  if (n_spec <= 0) return hipSuccess;
  return c->prec == SOAP_PREC_FP32 ? launch_t<float>(pl, c->P, n_spec, in, out, st)
                                   : launch_t<double>(pl, c->P, n_spec, in, out, st);
}

}  // namespace soap
