// Per-star kernels: disk-column Doppler shifts, chromatic contrast and the
// quiet integrated spectrum.
//
// Section 3.2 (Eqs. 5-11): on a log-uniform grid ln(lambda_m) = ln0 + m dln
// the relativistic factor of Eq. 6 is a translation by
// s = ln(1+f)/dln = atanh(beta)/dln pixels, the same for every pixel.  A disk
// column at x has beta = vsini x / c for all its cells (solid-body rotation),
// so the whole column shares one shift.  The bracketing index of Eqs. 9-10
// is n = m - ceil(s) and the interpolation factor of Eq. 11,
// (lambda_m - lambda'_n)/(lambda'_{n+1} - lambda'_n), evaluates exactly to
// w = expm1(u dln)/expm1(dln) with u = ceil(s) - s.  The shifted spectrum is
// S'_m = (1-w) S[m - c] + w S[m - c + 1] with the source index held inside
// [0, P-1] (end values held outside the shifted grid).
//
// Algorithm 1 (quiet disk): Q = sum over disk cells of A I(mu) S'_{q,bin}.
// Cells are summed per (column, mu bin) first ("column sums", FP32 + Kahan in
// the FP32 mode, FP64 otherwise, then one wave64 reduction in FP64), then the
// column sums are collapsed in FP64 onto integer offsets j:
//   K[b][j] = sum_{c_i = j} (1 - w_i) W[i][b] + sum_{c_i - 1 = j} w_i W[i][b]
// and Q[m] = sum_b sum_j K[b][j] S_{q,b}[clamp(m - j)], accumulated in FP64.
#include "soap_internal.hpp"

namespace soap {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

__global__ void k_geom(int N, double vsini, double dln, int* __restrict__ col_c,
                       double* __restrict__ col_w) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double x = cell_coord(i, N);
  double beta = vsini * x / C_KMS;
  double s = atanh(beta) / dln;
  double c = ceil(s);
  double u = c - s;
  col_c[i] = (int)c;
  col_w[i] = expm1(u * dln) / expm1(dln);
}

// contrast arrays over whole padded rows: pad entries hold the end values
template <typename T>
__global__ void k_contrast(int64_t P, int64_t Pstride, int B, double ln0, double dln, double teff, double dts,
                           double f0, double f1, double f2, const double* __restrict__ mu_b,
                           T* __restrict__ con_spot, T* __restrict__ con_fac) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // index in the padded row
  if (i >= Pstride) return;
  int64_t m = i - PAD_FRONT;
  m = m < 0 ? 0 : (m >= P ? P - 1 : m);
  double lam = exp(ln0 + dln * (double)m) * 1e-10;
  double eref = expm1(C2_MK / (lam * teff));
  con_spot[i] = (T)(eref / expm1(C2_MK / (lam * (teff - dts))));
  for (int b = 0; b < B; ++b) {
    double mu = mu_b[b];
    double dt = f0 + f1 * mu + f2 * mu * mu;
    con_fac[(int64_t)b * Pstride + i] = (T)(eref / expm1(C2_MK / (lam * (teff + dt))));
  }
}

template <typename T>
__global__ void k_fill_one(int64_t n, T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = T(1);
}

// fill the pads of every row with the row's first / last sample
template <typename T>
__global__ void k_pad(int64_t P, int64_t Pstride, int rows, T* __restrict__ base) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int row = blockIdx.y;
  if (row >= rows || i >= Pstride) return;
  T* r = base + (int64_t)row * Pstride;
  const int64_t m = i - PAD_FRONT;
  if (m < 0) r[i] = r[PAD_FRONT];
  else if (m >= P) r[i] = r[PAD_FRONT + P - 1];
}

// flags a non-finite value in `rows` padded rows (and optionally Q)
template <typename T>
__global__ void k_check_finite(int64_t n, const T* __restrict__ base, int64_t nq, const double* __restrict__ Q,
                               int* __restrict__ flag) {
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    bad = bad || !isfinite((double)base[i]);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += stride)
    bad = bad || !isfinite(Q[i]);
  if (bad) flag[0] = 1;
}

// one wave64 per disk column: W[i][b] = sum_{cells of column i in bin b} A I
template <bool KAHAN32>
__global__ void __launch_bounds__(64) k_quiet_colsum(int N, int B, double u1, double u2,
                                                     const double* __restrict__ mu_b,
                                                     double* __restrict__ colW) {
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const double x = cell_coord(i, N);
  const double area = (2.0 / N) * (2.0 / N);
  int bmin = B, bmax = -1;
  for (int k = lane; k < N; k += 64) {
    double y = cell_coord(k, N);
    double r2;
    {
#pragma clang fp contract(off)
      r2 = x * x + y * y;
    }
    if (r2 < 1.0) {
      int b = nearest_bin(sqrt(1.0 - r2), mu_b, B);
      bmin = min(bmin, b);
      bmax = max(bmax, b);
    }
  }
  bmin = wave_min(bmin);
  bmax = wave_max(bmax);
  for (int b = 0; b < B; ++b) {
    double tot = 0.0;
    if (b >= bmin && b <= bmax) {
      double part;
      if (KAHAN32) {
        float s = 0.f, comp = 0.f;
        for (int k = lane; k < N; k += 64) {
          double y = cell_coord(k, N);
          double r2;
          {
#pragma clang fp contract(off)
            r2 = x * x + y * y;
          }
          if (r2 < 1.0) {
            double mu = sqrt(1.0 - r2);
            if (nearest_bin(mu, mu_b, B) == b) {
              float v = (float)(area * limb_dark(mu, u1, u2));
              float yk = v - comp;
              float t = s + yk;
              comp = (t - s) - yk;
              s = t;
            }
          }
        }
        part = (double)s - (double)comp;
      } else {
        double s = 0.0;
        for (int k = lane; k < N; k += 64) {
          double y = cell_coord(k, N);
          double r2;
          {
#pragma clang fp contract(off)
            r2 = x * x + y * y;
          }
          if (r2 < 1.0) {
            double mu = sqrt(1.0 - r2);
            if (nearest_bin(mu, mu_b, B) == b) s += area * limb_dark(mu, u1, u2);
          }
        }
        part = s;
      }
      tot = wave_sum(part);
    }
    if (lane == 0) colW[(int64_t)i * B + b] = tot;
  }
}

// K[b][j] over columns in index order (FP64, deterministic)
__global__ void k_quiet_collapse(int N, int B, int jmin, int J, const int* __restrict__ col_c,
                                 const double* __restrict__ col_w, const double* __restrict__ colW,
                                 double* __restrict__ Kq) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * J) return;
  int b = t / J;
  int j = jmin + t % J;
  double acc = 0.0;
  for (int i = 0; i < N; ++i) {
    int c = col_c[i];
    double w = col_w[i];
    double W = colW[(int64_t)i * B + b];
    if (c == j) acc += (1.0 - w) * W;
    if (c - 1 == j) acc += w * W;
  }
  Kq[t] = acc;
}

// Differential rotation: quiet taps K[b][j] from per-cell shifts.  One wave
// per disk column; each visible cell splits A I(mu) onto its two offsets
// (Eq. 11) in an LDS table [B][J] of exact 64-bit fixed-point sums, which the
// wave adds to the global fixed-point table (order-free, so the totals repeat
// bit for bit).
__global__ void __launch_bounds__(64) k_quiet_dr(int N, int B, int J, int jmin, double u1, double u2,
                                                 double vsini, double diff_rot, double sin_i, double cos_i,
                                                 double dln, const double* __restrict__ mu_b,
                                                 unsigned long long* __restrict__ Kfx) {
  extern __shared__ unsigned long long s_q[];  // [B * J]
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const int BJ = B * J;
  for (int e = lane; e < BJ; e += 64) s_q[e] = 0ull;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const double x = cell_coord(i, N);
  const double area = (2.0 / N) * (2.0 / N);
  for (int k = lane; k < N; k += 64) {
    const double y = cell_coord(k, N);
    double r2;
    {
#pragma clang fp contract(off)
      r2 = x * x + y * y;
    }
    if (!(r2 < 1.0)) continue;
    const double mu = sqrt(1.0 - r2);
    const int b = nearest_bin(mu, mu_b, B);
    int cc;
    double w;
    cell_shift(x, y, mu, vsini, diff_rot, sin_i, cos_i, dln, &cc, &w);
    const int ja = cc - jmin, jb = cc - 1 - jmin;
    if (jb < 0 || ja >= J) continue;  // unreachable: the offset range bounds every shift
    const double aw = area * limb_dark(mu, u1, u2);
    atomicAdd(&s_q[b * J + ja], (unsigned long long)__double2ll_rn((1.0 - w) * aw * FX_ONE));
    atomicAdd(&s_q[b * J + jb], (unsigned long long)__double2ll_rn(w * aw * FX_ONE));
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int e = lane; e < BJ; e += 64) {
    const unsigned long long v = s_q[e];
    if (v) atomicAdd(Kfx + e, v);
  }
}

__global__ void k_quiet_dr_convert(int n, const unsigned long long* __restrict__ Kfx, double* __restrict__ Kq) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) Kq[t] = (double)(long long)Kfx[t] * FX_INV;
}

template <typename T>
__global__ void k_quiet(int64_t P, int64_t Pstride, int64_t Qlen, int B, int jmin, int J,
                        const double* __restrict__ Kq, const T* __restrict__ S, double* __restrict__ Q) {
  int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= Qlen) return;
  if (m >= P) {
    Q[m] = 0.0;
    return;
  }
  double acc = 0.0;
  for (int b = 0; b < B; ++b) {
    const T* row = S + (int64_t)b * Pstride;
    for (int jj = 0; jj < J; ++jj) {
      double k = Kq[b * J + jj];
      if (k != 0.0) {
        int64_t src = m - (jmin + jj);
        src = src < 0 ? 0 : (src >= P ? P - 1 : src);
        acc += k * (double)row[src];
      }
    }
  }
  Q[m] = acc;
}

template <typename T>
__global__ void k_q_convert(int64_t P, const double* __restrict__ Q, T* __restrict__ out) {
  int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m < P) out[m] = (T)Q[m];
}

hipError_t launch_geom(soap_ctx* c) {
  hipLaunchKernelGGL(k_geom, dim3((c->N + 255) / 256), dim3(256), 0, c->stream, c->N, c->vsini, c->dln,
                     c->d_col_c, c->d_col_w);
  return hipGetLastError();
}

hipError_t launch_contrast(soap_ctx* c) {
  dim3 grid((unsigned)((c->Pstride + 255) / 256));
  // the pointers address pixel 0; the kernel writes whole padded rows
  if (c->prec == SOAP_PREC_FP32)
    hipLaunchKernelGGL(k_contrast<float>, grid, dim3(256), 0, c->stream, c->P, c->Pstride, c->B, c->ln0, c->dln,
                       c->teff, c->dt_spot, c->dt_fac[0], c->dt_fac[1], c->dt_fac[2], c->d_mu,
                       (float*)c->d_con_spot - PAD_FRONT, (float*)c->d_con_fac - PAD_FRONT);
  else
    hipLaunchKernelGGL(k_contrast<double>, grid, dim3(256), 0, c->stream, c->P, c->Pstride, c->B, c->ln0, c->dln,
                       c->teff, c->dt_spot, c->dt_fac[0], c->dt_fac[1], c->dt_fac[2], c->d_mu,
                       (double*)c->d_con_spot - PAD_FRONT, (double*)c->d_con_fac - PAD_FRONT);
  return hipGetLastError();
}

hipError_t launch_ones(soap_ctx* c) {
  const int64_t n = (int64_t)c->n_tiles * APPLY_TILE_MAX;
  dim3 grid((unsigned)((n + 255) / 256));
  if (c->prec == SOAP_PREC_FP32)
    hipLaunchKernelGGL(k_fill_one<float>, grid, dim3(256), 0, c->stream, n, (float*)c->d_ones);
  else
    hipLaunchKernelGGL(k_fill_one<double>, grid, dim3(256), 0, c->stream, n, (double*)c->d_ones);
  return hipGetLastError();
}

hipError_t launch_pad(soap_ctx* c) {
  for (int t = 0; t < 3; ++t) {
    if (!c->d_spec_base[t]) continue;
    dim3 grid((unsigned)((c->Pstride + 255) / 256), c->B);
    if (c->prec == SOAP_PREC_FP32) {
      hipLaunchKernelGGL(k_pad<float>, grid, dim3(256), 0, c->stream, c->P, c->Pstride, c->B,
                         (float*)c->d_spec_base[t]);
    } else {
      hipLaunchKernelGGL(k_pad<double>, grid, dim3(256), 0, c->stream, c->P, c->Pstride, c->B,
                         (double*)c->d_spec_base[t]);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_pad_rows(soap_ctx* c, void* base, int rows) {
  if (!base || rows <= 0) return hipSuccess;
  dim3 grid((unsigned)((c->Pstride + 255) / 256), rows);
  if (c->prec == SOAP_PREC_FP32)
    hipLaunchKernelGGL(k_pad<float>, grid, dim3(256), 0, c->stream, c->P, c->Pstride, rows, (float*)base);
  else
    hipLaunchKernelGGL(k_pad<double>, grid, dim3(256), 0, c->stream, c->P, c->Pstride, rows, (double*)base);
  return hipGetLastError();
}

hipError_t launch_check_finite(soap_ctx* c, const void* base, int rows, bool with_q, int* d_flag) {
  const int64_t n = base ? (int64_t)rows * c->Pstride : 0;
  const int64_t nq = with_q ? (int64_t)c->n_tiles * APPLY_TILE_MAX : 0;
  if (n == 0 && nq == 0) return hipSuccess;
  const dim3 grid(1024), block(256);
  if (c->prec == SOAP_PREC_FP32)
    hipLaunchKernelGGL(k_check_finite<float>, grid, block, 0, c->stream, n, (const float*)base, nq, c->d_Q, d_flag);
  else
    hipLaunchKernelGGL(k_check_finite<double>, grid, block, 0, c->stream, n, (const double*)base, nq, c->d_Q,
                       d_flag);
  return hipGetLastError();
}

hipError_t launch_quiet(soap_ctx* c) {
  if (c->diff_rot != 0.0) {
    const int nt = c->B * c->J;
    hipLaunchKernelGGL(k_quiet_dr, dim3(c->N), dim3(64), (size_t)nt * sizeof(unsigned long long), c->stream, c->N,
                       c->B, c->J, c->jmin, c->u1, c->u2, c->vsini, c->diff_rot, c->sin_i, c->cos_i, c->dln, c->d_mu,
                       c->d_Kq_fx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_quiet_dr_convert, dim3((nt + 255) / 256), dim3(256), 0, c->stream, nt, c->d_Kq_fx, c->d_Kq);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t qlen = (int64_t)c->n_tiles * APPLY_TILE_MAX;
    dim3 grid((unsigned)((qlen + 255) / 256));
    if (c->prec == SOAP_PREC_FP32)
      hipLaunchKernelGGL(k_quiet<float>, grid, dim3(256), 0, c->stream, c->P, c->Pstride, qlen, c->B, c->jmin,
                         c->J, c->d_Kq, (const float*)c->d_spec[SOAP_QUIET], c->d_Q);
    else
      hipLaunchKernelGGL(k_quiet<double>, grid, dim3(256), 0, c->stream, c->P, c->Pstride, qlen, c->B, c->jmin,
                         c->J, c->d_Kq, (const double*)c->d_spec[SOAP_QUIET], c->d_Q);
    return hipGetLastError();
  }
  if (c->prec == SOAP_PREC_FP32)
    hipLaunchKernelGGL(k_quiet_colsum<true>, dim3(c->N), dim3(64), 0, c->stream, c->N, c->B, c->u1, c->u2,
                       c->d_mu, c->d_colW);
  else
    hipLaunchKernelGGL(k_quiet_colsum<false>, dim3(c->N), dim3(64), 0, c->stream, c->N, c->B, c->u1, c->u2,
                       c->d_mu, c->d_colW);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int nt = c->B * c->J;
  hipLaunchKernelGGL(k_quiet_collapse, dim3((nt + 255) / 256), dim3(256), 0, c->stream, c->N, c->B, c->jmin,
                     c->J, c->d_col_c, c->d_col_w, c->d_colW, c->d_Kq);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t qlen = (int64_t)c->n_tiles * APPLY_TILE_MAX;
  dim3 grid((unsigned)((qlen + 255) / 256));
  if (c->prec == SOAP_PREC_FP32)
    hipLaunchKernelGGL(k_quiet<float>, grid, dim3(256), 0, c->stream, c->P, c->Pstride, qlen, c->B, c->jmin,
                       c->J, c->d_Kq, (const float*)c->d_spec[SOAP_QUIET], c->d_Q);
  else
    hipLaunchKernelGGL(k_quiet<double>, grid, dim3(256), 0, c->stream, c->P, c->Pstride, qlen, c->B, c->jmin,
                       c->J, c->d_Kq, (const double*)c->d_spec[SOAP_QUIET], c->d_Q);
  return hipGetLastError();
}

hipError_t launch_q_convert(soap_ctx* c, void* out) {
  dim3 grid((unsigned)((c->P + 255) / 256));
  hipLaunchKernelGGL(k_q_convert<float>, grid, dim3(256), 0, c->stream, c->P, c->d_Q, (float*)out);
  return hipGetLastError();
}

}  // namespace soap
