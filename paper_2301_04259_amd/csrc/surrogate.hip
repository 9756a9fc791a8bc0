// Learned surrogate of the disk-integrated spectrum: a small MLP that maps
// the active-region and star parameters of one spectrum to the PCA
// coefficients of its difference from the quiet spectrum (Eqs. 1-4 give the
// spectrum the network stands in for), with its training and inference
// kernels.
//
// Network per ensemble member: x[n_in] -> SiLU(x W1 + b1)[H] ->
// SiLU(. W2 + b2)[H] -> . W3 + b3 [n_out].  Parameters are FP32 masters;
// the matrix products run on BF16 copies with MFMA (v_mfma_f32_16x16x32_bf16,
// FP32 accumulate), one 16 x 16 output tile per wave.  Training minimises the
// mean squared error over the batch and outputs with Adam (bias-corrected
// moments, FP32).  Every kernel has a fixed order of operations, so results
// repeat bit for bit.
//
// The PCA projection coef = (d - mean) V of spectra differences onto a basis
// is an FP32 tiled product (K = pixels, large).
#include <cmath>

#include "surrogate_internal.hpp"
#include "wave.hpp"

namespace soap {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }

__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

}  // namespace

// C[M][N] = op(A)[M][K] op(B)[K][N] for every ensemble member (grid z), BF16
// in, FP32 accumulate.  op(A)(i, k) = TA ? A[k lda + i] : A[i lda + k];
// op(B)(k, j) = TB ? B[j ldb + k] : B[k ldb + j].  M, N multiples of 16, K a
// multiple of 32, lda and ldb multiples of 8 (16-byte rows of 8 elements).
// A block of four waves computes a 64 x 64 tile of C, each wave a 32 x 32
// quarter as 2 x 2 MFMA tiles of 16 x 16 (v_mfma_f32_16x16x32_bf16: lane l
// holds A(l % 16, 8 (l / 16) + e) and B(8 (l / 16) + e, l % 16), e < 8, and
// ends with C(4 (l / 16) + r, l % 16), r < 4).  Per K step of 32 the block
// stages the 64 x 32 slices of op(A) and op(B)^T in LDS with 16-byte global
// loads (one per thread and operand), so every lane reads its 8 operands as
// one 16-byte LDS read; rows past M or N read a clamped row and are not
// stored.  Each output adds its K steps in order, as one MFMA chain.
constexpr int MM_T = 64;        // block tile
constexpr int MM_LDK = 32 + 8;  // LDS row of 32 k values, padded against bank conflicts

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) k_mm_bf16(int M, int N, int K, const __bf16* __restrict__ A, int lda,
                                                 int64_t sA, const __bf16* __restrict__ B, int ldb, int64_t sB,
                                                 const float* __restrict__ bias, int64_t sBias, float* __restrict__ Cf,
                                                 int ldc, int64_t sC, __bf16* __restrict__ Cb, int64_t sCb,
                                                 const float* __restrict__ Z, int64_t sZ) {
  __shared__ __align__(16) __bf16 As[MM_T][MM_LDK];  // op(A) rows i, k contiguous
  __shared__ __align__(16) __bf16 Bs[MM_T][MM_LDK];  // op(B) columns j, k contiguous
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int i0 = blockIdx.y * MM_T, j0 = blockIdx.x * MM_T;
  const int e_ = blockIdx.z;
  A += e_ * sA;
  B += e_ * sB;
  // staging: thread t moves 8 elements of each operand per K step
  //   k-contiguous source: row t / 4 of the tile, k = 8 (t % 4) .. + 8
  //   row-contiguous source: k = t / 8, rows 8 (t % 8) .. + 8
  const int r_kc = t >> 2, k_kc = 8 * (t & 3);
  const int k_rc = t >> 3, r_rc = 8 * (t & 7);
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    if (k0) __syncthreads();  // every wave is done with the previous slices
    if constexpr (!TA) {
      const int i = min(i0 + r_kc, M - 1);
      *reinterpret_cast<bf16x8*>(&As[r_kc][k_kc]) =
          *reinterpret_cast<const bf16x8*>(A + (int64_t)i * lda + k0 + k_kc);
    } else {
      const int i = min(i0 + r_rc, M - 8);  // M is a multiple of 16, so the 8 rows stay in range
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(A + (int64_t)(k0 + k_rc) * lda + i);
#pragma unroll
      for (int e = 0; e < 8; ++e) As[i - i0 + e < MM_T ? i - i0 + e : MM_T - 1][k_rc] = v[e];
    }
    if constexpr (TB) {
      const int j = min(j0 + r_kc, N - 1);
      *reinterpret_cast<bf16x8*>(&Bs[r_kc][k_kc]) =
          *reinterpret_cast<const bf16x8*>(B + (int64_t)j * ldb + k0 + k_kc);
    } else {
      const int j = min(j0 + r_rc, N - 8);
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(B + (int64_t)(k0 + k_rc) * ldb + j);
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[j - j0 + e < MM_T ? j - j0 + e : MM_T - 1][k_rc] = v[e];
    }
    __syncthreads();
    bf16x8 av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * a + (l & 15)][8 * (l >> 4)]);
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * b + (l & 15)][8 * (l >> 4)]);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = j0 + wn + 16 * b + (l & 15);
      if (j >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm + 16 * a + 4 * (l >> 4) + r;
        if (i >= M) continue;
        const int64_t o = (int64_t)i * ldc + j;
        const float v = acc[a][b][r];
        if constexpr (EPI == MM_HIDDEN) {  // z = v + b, keep z, emit SiLU(z) in BF16
          const float z = v + bias[e_ * sBias + j];
          Cf[e_ * sC + o] = z;
          Cb[e_ * sCb + o] = (__bf16)silu(z);
        } else if constexpr (EPI == MM_OUTPUT) {  // y = v + b
          Cf[e_ * sC + o] = v + bias[e_ * sBias + j];
        } else if constexpr (EPI == MM_DHIDDEN) {  // dz = v SiLU'(z), in FP32 and BF16
          const float dz = v * silu_grad(Z[e_ * sZ + o]);
          Cf[e_ * sC + o] = dz;
          Cb[e_ * sCb + o] = (__bf16)dz;
        } else {  // MM_PLAIN: weight gradient
          Cf[e_ * sC + o] = v;
        }
      }
    }
}

// x[B][n_in] (FP32) -> X[B][K0] (BF16, zero padded)
__global__ void k_pack_input(int B, int n_in, int K0, const float* __restrict__ x, __bf16* __restrict__ X) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * K0) return;
  const int i = (int)(t / K0), k = (int)(t - (int64_t)i * K0);
  X[t] = (__bf16)(k < n_in ? x[(int64_t)i * n_in + k] : 0.f);
}

// Squared error per (member, row) and dY = 2 (y - t) / (B n_out) in BF16: one
// wave per row (lanes over outputs, fixed-order wave sum), four rows a block
__global__ void __launch_bounds__(256) k_mse(int B, int n_out, const float* __restrict__ Y,
                                             const float* __restrict__ T, __bf16* __restrict__ dY,
                                             float* __restrict__ row_se) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int e = blockIdx.y;
  if (i >= B) return;  // whole wave
  const float sc = 2.0f / ((float)B * (float)n_out);
  const float* y = Y + ((int64_t)e * B + i) * n_out;
  const float* t = T + (int64_t)i * n_out;
  __bf16* d = dY + ((int64_t)e * B + i) * n_out;
  float se = 0.f;
  for (int j = lane; j < n_out; j += 64) {
    const float df = y[j] - t[j];
    se = fmaf(df, df, se);
    d[j] = (__bf16)(sc * df);
  }
  const double tot = wave_sum_f64((double)se);
  if (lane == 0) row_se[(int64_t)e * B + i] = (float)tot;
}

// per member: loss = sum of row_se / (B n_out), rows added in order by one
// block of 256 threads (strided partials, then a fixed tree)
__global__ void __launch_bounds__(256) k_loss_sum(int B, int n_out, const float* __restrict__ row_se,
                                                  float* __restrict__ loss) {
  __shared__ float s[256];
  const int e = blockIdx.x;
  float a = 0.f;
  for (int i = threadIdx.x; i < B; i += 256) a += row_se[(int64_t)e * B + i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[e] = s[0] / ((float)B * (float)n_out);
}

// db[j] = sum_i D[i][j] per member, in two fixed-order stages: partial sums
// over chunks of SG_COLSUM_ROWS rows (block: 64 columns x 4 row phases,
// combined in phase order), then the chunks in order
__global__ void __launch_bounds__(256) k_colsum_part(int B, int N, const float* __restrict__ D, int64_t sD,
                                                     float* __restrict__ part) {
  __shared__ float s[4][64];
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;
  const int c = blockIdx.y, e = blockIdx.z;
  const int r0 = c * SG_COLSUM_ROWS, r1 = min(B, r0 + SG_COLSUM_ROWS);
  float a = 0.f;
  if (col < N)
    for (int i = r0 + g; i < r1; i += 4) a += D[e * sD + (int64_t)i * N + col];
  s[g][threadIdx.x & 63] = a;
  __syncthreads();
  if (g == 0 && col < N) {
    const int l = threadIdx.x;
    part[((int64_t)e * gridDim.y + c) * N + col] = ((s[0][l] + s[1][l]) + s[2][l]) + s[3][l];
  }
}

__global__ void k_colsum_final(int n_chunks, int N, const float* __restrict__ part, float* __restrict__ db,
                               int64_t sdb) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = blockIdx.y;
  if (j >= N) return;
  float a = 0.f;
  for (int c = 0; c < n_chunks; ++c) a += part[((int64_t)e * n_chunks + c) * N + j];
  db[e * sdb + j] = a;
}

// dY (BF16) -> FP32 copy for the output-bias gradient
__global__ void k_bf16_to_f32(int64_t n, const __bf16* __restrict__ a, float* __restrict__ b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = (float)a[t];
}

// Adam on the FP32 masters (all members), then the BF16 copies
__global__ void k_adam(int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       float* __restrict__ P, const float* __restrict__ G, float* __restrict__ Mm,
                       float* __restrict__ Vm, __bf16* __restrict__ Pb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float g = G[t];
  const float m = b1 * Mm[t] + (1.0f - b1) * g;
  const float v = b2 * Vm[t] + (1.0f - b2) * g * g;
  Mm[t] = m;
  Vm[t] = v;
  const float mh = m / c1, vh = v / c2;
  const float p = P[t] - lr * mh / (sqrtf(vh) + eps);
  P[t] = p;
  Pb[t] = (__bf16)p;
}

__global__ void k_f32_to_bf16(int64_t n, const float* __restrict__ a, __bf16* __restrict__ b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = (__bf16)a[t];
}

// ensemble mean of the outputs (members added in order)
__global__ void k_ens_mean(int64_t n, int E, const float* __restrict__ Y, float* __restrict__ mean) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  float m = 0.f;
  for (int e = 0; e < E; ++e) m += Y[(int64_t)e * n + t];
  mean[t] = m / (float)E;
}

// per sample: RV of the mean prediction, calib x sample standard deviation
// of the members' RVs, and the fallback flag
__global__ void k_gate(int64_t n, int E, double calib, double thr, const soap_rv* __restrict__ rv,
                       double* __restrict__ rv_kms, double* __restrict__ err_kms, int* __restrict__ fallback) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool bad = rv[i].status != 0;
  double m = 0.0;
  for (int e = 0; e < E; ++e) {
    const soap_rv& r = rv[(1 + e) * n + i];
    bad = bad || r.status != 0;
    m += r.rv_kms;
  }
  m /= (double)E;
  double v = 0.0;
  for (int e = 0; e < E; ++e) {
    const double d = rv[(1 + e) * n + i].rv_kms - m;
    v += d * d;
  }
  const double err = calib * sqrt(v / (double)(E - 1));
  rv_kms[i] = rv[i].rv_kms;
  if (err_kms) err_kms[i] = err;
  fallback[i] = (bad || !(err < thr)) ? 1 : 0;
}

// coef[n][k] = sum_p (D[n][p] - mean[p]) V[p][k] (mean row mean_idx[n] when
// given): 64 x 64 tile per block of
// 256 threads (4 x 4 outputs each), K in steps of 32 through LDS, FP32
// Network inputs of one sample from its raw description r = (lat, lon,
// radius, contrast, phase, T_eff, inclination, v sin i) in degrees, R*, K
// and km/s: the spot latitude scaled to +-60 deg, the sine and cosine of
// its rotated longitude, its centre on the sky (x, y, z; y up the projected
// axis, z towards the observer), and the scalar parameters centred and
// scaled over their sampled ranges, then a constant 1.
__global__ void __launch_bounds__(256) k_features(int64_t n, const double* __restrict__ raw, float* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* r = raw + i * SG_RAW;
  constexpr double D2R = 3.14159265358979323846 / 180.0;
  const double lat = r[0] * D2R;
  const double th = (r[1] + 360.0 * r[4]) * D2R;
  const double inc = r[6] * D2R;
  const double cl = cos(lat), sl = sin(lat), st = sin(th), ct = cos(th), si = sin(inc), ci = cos(inc);
  float* o = x + i * SG_FEATURES;
  o[0] = (float)(lat / (60.0 * D2R));
  o[1] = (float)st;
  o[2] = (float)ct;
  o[3] = (float)(cl * st);
  o[4] = (float)(sl * si - cl * ct * ci);
  o[5] = (float)(sl * ci + cl * ct * si);
  o[6] = (float)((r[2] - 0.055) / 0.045);
  o[7] = (float)((r[3] - 0.6) / 0.3);
  o[8] = (float)((r[5] - 5500.0) / 1000.0);
  o[9] = (float)((r[6] - 60.0) / 30.0);
  o[10] = (float)((r[7] - 3.0) / 2.0);
  o[11] = 1.0f;
}

__global__ void __launch_bounds__(256) k_pca_project(int n, int P, int k, const float* __restrict__ D,
                                                     int64_t ldd, const float* __restrict__ mean,
                                                     const int* __restrict__ mean_idx, int n_mean,
                                                     const float* __restrict__ V, float* __restrict__ coef) {
  __shared__ float sA[32][64 + 1];
  __shared__ float sB[32][64 + 1];
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;  // rows on x: up to 2^25 / 64 blocks
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  float acc[4][4] = {};
  for (int p0 = 0; p0 < P; p0 += 32) {
    for (int t = threadIdx.x; t < 32 * 64; t += 256) {
      const int pp = t & 31, rr = t >> 5;  // A: row rr, pixel pp (coalesced over pixels)
      const int row = r0 + rr, pix = p0 + pp;
      int mi = (mean_idx && row < n) ? mean_idx[row] : 0;
      const bool bad = mi < 0 || mi >= n_mean;  // no such centre: the row's coefficients are NaN
      mi = bad ? 0 : mi;
      const float* mrow = mean + (int64_t)mi * P;
      sA[pp][rr] = (row < n && pix < P) ? (bad ? __builtin_nanf("") : D[(int64_t)row * ldd + pix] - mrow[pix]) : 0.f;
      const int cc = t & 63, pq = t >> 6;  // B: pixel pq < 32, component cc
      const int pb = p0 + pq, col = c0 + cc;
      sB[pq][cc] = (pb < P && col < k) ? V[(int64_t)pb * k + col] : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int pp = 0; pp < 32; ++pp) {
      float a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = sA[pp][ty * 4 + u];
        b[u] = sB[pp][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[u][w] = fmaf(a[u], b[w], acc[u][w]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int row = r0 + ty * 4 + u, col = c0 + tx * 4 + w;
      if (row < n && col < k) coef[(int64_t)row * k + col] = acc[u][w];
    }
}

// ---- launchers -------------------------------------------------------------

namespace {

template <bool TA, bool TB, int EPI>
hipError_t mm(hipStream_t st, int E, int M, int N, int K, const __bf16* A, int lda, int64_t sA, const __bf16* B,
              int ldb, int64_t sB, const float* bias, int64_t sBias, float* Cf, int ldc, int64_t sC, __bf16* Cb,
              int64_t sCb, const float* Z, int64_t sZ) {
  if (M % 16 || N % 16 || K % 32 || lda % 8 || ldb % 8) return hipErrorInvalidValue;
  dim3 grid((N + MM_T - 1) / MM_T, (M + MM_T - 1) / MM_T, E);
  hipLaunchKernelGGL((k_mm_bf16<TA, TB, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, sA, B, ldb, sB, bias,
                     sBias, Cf, ldc, sC, Cb, sCb, Z, sZ);
  return hipGetLastError();
}

inline dim3 blocks(int64_t n, int t = 256) { return dim3((unsigned)((n + t - 1) / t)); }

hipError_t colsum(hipStream_t st, int E, int B, int N, const float* D, int64_t sD, float* part, float* db,
                  int64_t sdb) {
  const int nc = (B + SG_COLSUM_ROWS - 1) / SG_COLSUM_ROWS;
  hipLaunchKernelGGL(k_colsum_part, dim3((N + 63) / 64, nc, E), dim3(256), 0, st, B, N, D, sD, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum_final, dim3((N + 255) / 256, E), dim3(256), 0, st, nc, N, part, db, sdb);
  return hipGetLastError();
}

}  // namespace

#define SG_TRY(x)                              \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return e_;           \
  } while (0)

hipError_t sg_forward(soap_surrogate* s, const float* x, int B) {
  const SgLayout& L = s->lay;
  const int E = s->n_ens, H = s->hidden;
  hipStream_t st = s->stream;
  hipLaunchKernelGGL(k_pack_input, blocks((int64_t)B * SG_K0), dim3(256), 0, st, B, s->n_in, SG_K0, x, s->X);
  SG_TRY(hipGetLastError());
  const int64_t sP = L.n_params;
  // layer 1: K0 -> H
  SG_TRY((mm<false, false, MM_HIDDEN>(st, E, B, H, SG_K0, s->X, SG_K0, 0, s->Pb + L.W1, H, sP, s->P + L.b1, sP,
                                      s->Z1, H, (int64_t)B * H, s->H1, (int64_t)B * H, nullptr, 0)));
  // layer 2: H -> H
  SG_TRY((mm<false, false, MM_HIDDEN>(st, E, B, H, H, s->H1, H, (int64_t)B * H, s->Pb + L.W2, H, sP, s->P + L.b2,
                                      sP, s->Z2, H, (int64_t)B * H, s->H2, (int64_t)B * H, nullptr, 0)));
  // layer 3: H -> n_out
  SG_TRY((mm<false, false, MM_OUTPUT>(st, E, B, s->n_out, H, s->H2, H, (int64_t)B * H, s->Pb + L.W3, s->n_out, sP,
                                      s->P + L.b3, sP, s->Y, s->n_out, (int64_t)B * s->n_out, nullptr, 0, nullptr,
                                      0)));
  return hipSuccess;
}

hipError_t sg_backward(soap_surrogate* s, const float* target, int B) {
  const SgLayout& L = s->lay;
  const int E = s->n_ens, H = s->hidden, O = s->n_out;
  hipStream_t st = s->stream;
  const int64_t sP = L.n_params, sBH = (int64_t)B * H, sBO = (int64_t)B * O;
  hipLaunchKernelGGL(k_mse, dim3((B + 3) / 4, E), dim3(256), 0, st, B, O, s->Y, target, s->dY, s->row_se);
  SG_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_loss_sum, dim3(E), dim3(256), 0, st, B, O, s->row_se, s->loss);
  SG_TRY(hipGetLastError());
  // output layer: dW3 = H2^T dY, db3 = colsum dY
  SG_TRY((mm<true, false, MM_PLAIN>(st, E, H, O, B, s->H2, H, sBH, s->dY, O, sBO, nullptr, 0, s->G + L.W3, O, sP,
                                    nullptr, 0, nullptr, 0)));
  hipLaunchKernelGGL(k_bf16_to_f32, blocks((int64_t)E * B * O), dim3(256), 0, st, (int64_t)E * B * O, s->dY,
                     s->dYf);
  SG_TRY(hipGetLastError());
  SG_TRY(colsum(st, E, B, O, s->dYf, sBO, s->colpart, s->G + L.b3, sP));
  // dZ2 = (dY W3^T) SiLU'(Z2); dW2 = H1^T dZ2; db2 = colsum dZ2
  SG_TRY((mm<false, true, MM_DHIDDEN>(st, E, B, H, O, s->dY, O, sBO, s->Pb + L.W3, O, sP, nullptr, 0, s->dZf, H, sBH,
                                      s->dZb, sBH, s->Z2, sBH)));
  SG_TRY((mm<true, false, MM_PLAIN>(st, E, H, H, B, s->H1, H, sBH, s->dZb, H, sBH, nullptr, 0, s->G + L.W2, H, sP,
                                    nullptr, 0, nullptr, 0)));
  SG_TRY(colsum(st, E, B, H, s->dZf, sBH, s->colpart, s->G + L.b2, sP));
  // dZ1 = (dZ2 W2^T) SiLU'(Z1); dW1 = X^T dZ1; db1 = colsum dZ1
  SG_TRY((mm<false, true, MM_DHIDDEN>(st, E, B, H, H, s->dZb, H, sBH, s->Pb + L.W2, H, sP, nullptr, 0, s->dZf2, H,
                                      sBH, s->dZb2, sBH, s->Z1, sBH)));
  SG_TRY((mm<true, false, MM_PLAIN>(st, E, SG_K0, H, B, s->X, SG_K0, 0, s->dZb2, H, sBH, nullptr, 0, s->G + L.W1, H,
                                    sP, nullptr, 0, nullptr, 0)));
  return colsum(st, E, B, H, s->dZf2, sBH, s->colpart, s->G + L.b1, sP);
}

hipError_t sg_adam(soap_surrogate* s, float lr) {
  s->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - powf(b1, (float)s->step), c2 = 1.0f - powf(b2, (float)s->step);
  const int64_t n = (int64_t)s->n_ens * s->lay.n_params;
  hipLaunchKernelGGL(k_adam, blocks(n), dim3(256), 0, s->stream, n, lr, b1, b2, eps, c1, c2, s->P, s->G, s->M, s->V,
                     s->Pb);
  return hipGetLastError();
}

hipError_t sg_sync_bf16(soap_surrogate* s) {
  const int64_t n = (int64_t)s->n_ens * s->lay.n_params;
  hipLaunchKernelGGL(k_f32_to_bf16, blocks(n), dim3(256), 0, s->stream, n, s->P, s->Pb);
  return hipGetLastError();
}

hipError_t sg_ens_mean(soap_surrogate* s, int B, float* mean) {
  const int64_t n = (int64_t)B * s->n_out;
  hipLaunchKernelGGL(k_ens_mean, blocks(n), dim3(256), 0, s->stream, n, s->n_ens, s->Y, mean);
  return hipGetLastError();
}

hipError_t sg_gate(hipStream_t st, const soap_rv* rv, int64_t n, int E, double calib, double thr, double* rv_kms,
                   double* err_kms, int* fallback) {
  hipLaunchKernelGGL(k_gate, blocks(n), dim3(256), 0, st, n, E, calib, thr, rv, rv_kms, err_kms, fallback);
  return hipGetLastError();
}

hipError_t sg_features(hipStream_t st, int64_t n, const double* raw, float* x) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, raw, x);
  return hipGetLastError();
}

hipError_t sg_pca_project(hipStream_t st, int n, int P, int k, const float* D, int64_t ldd, const float* mean,
                          const int* mean_idx, int n_mean, const float* V, float* coef) {
  dim3 grid((n + 63) / 64, (k + 63) / 64);
  hipLaunchKernelGGL(k_pca_project, grid, dim3(256), 0, st, n, P, k, D, ldd, mean, mean_idx,
                     mean_idx ? n_mean : 1, V, coef);
  return hipGetLastError();
}

}  // namespace soap
