// CCF against a line mask and Gaussian fit of the CCF (section 4.1: RVs from
// cross-correlation with a line mask and the mean of a fitted Gaussian).
//
// CCF: pixel m is a constant-flux bin [m, m+1) in the pixel coordinate
// q = (ln(lambda) - ln0)/dln + 1/2.  Mask line l sits at u_l in that
// coordinate; at trial velocity v_k its hole spans [u_l + a_k^-, u_l + a_k^+]
// with a_k^+- = atanh((v_k +- h)/c)/dln (the ln of the Eq. 6 factor).
// CCF_k = sum_l w_l sum_m F_m * overlap(bin m, hole), existing pixels only.
// Layout: one block per (block of lines, block of SB spectra), one thread per
// velocity; each thread keeps SB double accumulators and reuses its hole
// geometry for every spectrum of the block.  Partial sums per line block are
// added in a fixed order by a second kernel, so results repeat bit for bit.
//
// Fit: one wave64 per CCF; Levenberg-Marquardt in double on the unweighted
// least squares of c0 - a exp(-(v - mu)^2 / (2 sigma^2)); J^T J and J^T r
// are wave reductions, the 4 x 4 damped system is solved by Cholesky in every
// lane.  Start values: c0 = max, a = c0 - min, mu = v at the min, sigma from
// the half-depth width.
#include "soap_internal.hpp"

namespace soap {

constexpr int CCF_LINES = 64;  // lines per block (partial sums per block)
constexpr int CCF_BATCH = 16;  // lines staged in LDS at a time
constexpr int CCF_SB = 8;      // spectra per block
constexpr int CCF_THREADS = 192;
constexpr int CCF_LDS = 32768; // bytes of staged spectra per block
template <typename T>
constexpr int ccf_span() { return CCF_LDS / (CCF_SB * (int)sizeof(T)); }  // pixels per spectrum

int ccf_line_blocks(int n_lines) { return (n_lines + CCF_LINES - 1) / CCF_LINES; }
int ccf_span_pixels(bool fp32) { return fp32 ? ccf_span<float>() : ccf_span<double>(); }

__global__ void k_mask_prep(int n, double ln0, double dln, const double* __restrict__ lnl,
                            const double* __restrict__ w, double2* __restrict__ out) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < n) out[l] = make_double2((lnl[l] - ln0) / dln + 0.5, w[l]);
}

// One block per (64 mask lines, 8 spectra).  Lines are taken in batches of
// up to 16 whose holes, at any trial velocity, reach a pixel span that fits
// the LDS stage; that span is staged for the block's spectra (coalesced
// loads), then one thread per velocity computes each hole's pixel overlaps
// once and applies them to every staged spectrum, accumulating in double.
template <typename T>
__global__ void __launch_bounds__(CCF_THREADS) k_ccf(int64_t P, int64_t n_spec, const T* __restrict__ F,
                                                     int n_lines, const double2* __restrict__ mask, int n_v,
                                                     double v0, double dv, double h, double dln,
                                                     double* __restrict__ part) {
  constexpr int SPAN = ccf_span<T>();
  __shared__ T st[CCF_SB][SPAN];
  __shared__ int64_t s_lo;
  __shared__ int s_len, s_b1;
  const int lb = blockIdx.x;
  const int64_t s0 = (int64_t)blockIdx.y * CCF_SB;
  const int l0 = lb * CCF_LINES;
  const int l1 = min(n_lines, l0 + CCF_LINES);
  const int ns = (int)min<int64_t>(CCF_SB, n_spec - s0);
  // hole edges of every velocity this block handles: a thread keeps its own
  const int kk = threadIdx.x;  // velocities kk, kk + blockDim.x, ...
  // extreme edges over the velocity grid bound the staged span
  const double alo_min = atanh((v0 - h) / C_KMS) / dln;
  const double ahi_max = atanh((v0 + dv * (n_v - 1) + h) / C_KMS) / dln;
  double acc[4][CCF_SB];  // up to 4 velocities per thread (n_v <= 4 * CCF_THREADS)
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int s = 0; s < CCF_SB; ++s) acc[a][s] = 0.0;
  double alo[4], ahi[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int k = kk + a * CCF_THREADS;
    const double vk = v0 + dv * k;
    alo[a] = atanh((vk - h) / C_KMS) / dln;
    ahi[a] = atanh((vk + h) / C_KMS) / dln;
  }
  for (int b0 = l0; b0 < l1;) {
    if (threadIdx.x == 0) {
      // grow the batch while the reach of all its holes fits the stage
      int64_t lo = (int64_t)floor(mask[b0].x + alo_min);
      int64_t hi = (int64_t)floor(mask[b0].x + ahi_max) + 1;
      int e = b0 + 1;
      while (e < l1 && e - b0 < CCF_BATCH) {
        const int64_t nlo = min(lo, (int64_t)floor(mask[e].x + alo_min));
        const int64_t nhi = max(hi, (int64_t)floor(mask[e].x + ahi_max) + 1);
        if (nhi - nlo + 1 > SPAN) break;
        lo = nlo;
        hi = nhi;
        ++e;
      }
      s_lo = lo;
      s_len = (int)min<int64_t>(SPAN, hi - lo + 1);
      s_b1 = e;
    }
    __syncthreads();
    const int64_t lo = s_lo;
    const int len = s_len;
    const int b1 = s_b1;
    for (int s = 0; s < ns; ++s) {
      const T* row = F + (s0 + s) * P;
      for (int i = threadIdx.x; i < len; i += blockDim.x) {
        const int64_t m = lo + i;
        st[s][i] = (m >= 0 && m < P) ? row[m] : T(0);
      }
    }
    __syncthreads();
    for (int l = b0; l < b1; ++l) {
      const double2 mw = mask[l];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int k = kk + a * CCF_THREADS;
        if (k >= n_v) break;
        const double qlo = mw.x + alo[a];
        const double qhi = mw.x + ahi[a];
        const int64_t ma = (int64_t)floor(qlo);
        const int64_t mb = (int64_t)floor(qhi);
        for (int64_t m = ma; m <= mb; ++m) {
          const double ov = fmin(qhi, (double)(m + 1)) - fmax(qlo, (double)m);
          const int64_t i = m - lo;
          if (ov > 0.0 && m >= 0 && m < P && i >= 0 && i < len) {
            const double wo = mw.y * ov;
#pragma unroll
            for (int s = 0; s < CCF_SB; ++s) acc[a][s] = fma(wo, (double)st[s][i], acc[a][s]);
          }
        }
      }
    }
    __syncthreads();
    b0 = b1;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int k = kk + a * CCF_THREADS;
    if (k >= n_v) break;
#pragma unroll
    for (int s = 0; s < CCF_SB; ++s)
      if (s < ns) part[((int64_t)lb * n_spec + s0 + s) * n_v + k] = acc[a][s];
  }
}

__global__ void k_ccf_reduce(int n_lb, int64_t n_spec, int n_v, const double* __restrict__ part,
                             double* __restrict__ ccf) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_spec * n_v) return;
  double s = 0.0;
  for (int lb = 0; lb < n_lb; ++lb) s += part[(int64_t)lb * n_spec * n_v + t];
  ccf[t] = s;
}

namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr double FWHM_PER_SIGMA = 2.3548200450309493;  // 2 sqrt(2 ln 2)
constexpr int GF_MAXPT = 12;                            // points per lane (n_v <= 768)

// chi^2 and optionally J^T J (10 unique) / J^T r (4) at p
__device__ void gf_eval(const double* y, int n_v, double v0, double dv, const double p[4], bool jac,
                        double& chi2, double jtj[10], double jtr[4]) {
  const int lane = threadIdx.x;
  double c2 = 0.0;
  double a[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  double b[4] = {0, 0, 0, 0};
  const double is2 = 1.0 / (p[3] * p[3]);
  for (int t = 0; t < GF_MAXPT; ++t) {
    const int i = lane + 64 * t;
    if (i >= n_v) break;
    const double v = v0 + dv * i;
    const double d = v - p[2];
    const double e = exp(-0.5 * d * d * is2);
    const double r = p[0] - p[1] * e - y[i];
    c2 += r * r;
    if (jac) {
      const double g0 = 1.0;
      const double g1 = -e;
      const double g2 = -p[1] * e * d * is2;
      const double g3 = -p[1] * e * d * d * is2 / p[3];
      const double g[4] = {g0, g1, g2, g3};
      int q = 0;
      for (int r0 = 0; r0 < 4; ++r0) {
        b[r0] += g[r0] * r;
        for (int r1 = r0; r1 < 4; ++r1) a[q++] += g[r0] * g[r1];
      }
    }
  }
  chi2 = wsum(c2);
  if (jac) {
    for (int q = 0; q < 10; ++q) jtj[q] = wsum(a[q]);
    for (int q = 0; q < 4; ++q) jtr[q] = wsum(b[q]);
  }
}

// solve (A + lam diag A) x = -g for symmetric positive definite 4 x 4 A
__device__ bool gf_solve(const double jtj[10], const double jtr[4], double lam, double x[4]) {
  double A[4][4];
  int q = 0;
  for (int r0 = 0; r0 < 4; ++r0)
    for (int r1 = r0; r1 < 4; ++r1) {
      A[r0][r1] = jtj[q];
      A[r1][r0] = jtj[q];
      ++q;
    }
  for (int r = 0; r < 4; ++r) A[r][r] *= (1.0 + lam);
  double L[4][4] = {{0}};
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[i][i] = sqrt(s);
      } else {
        L[i][j] = s / L[j][j];
      }
    }
  }
  double z[4];
  for (int i = 0; i < 4; ++i) {
    double s = -jtr[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * z[k];
    z[i] = s / L[i][i];
  }
  for (int i = 3; i >= 0; --i) {
    double s = z[i];
    for (int k = i + 1; k < 4; ++k) s -= L[k][i] * x[k];
    x[i] = s / L[i][i];
  }
  return true;
}

}  // namespace

__global__ void __launch_bounds__(64) k_gfit(int64_t n_spec, int n_v, double v0, double dv,
                                             const double* __restrict__ ccf, soap_rv* __restrict__ out) {
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  const double* y = ccf + s * n_v;
  // start values: max, first argmin, half-depth width
  double ymax = -1e308, ymin = 1e308;
  int kmin = n_v;
  for (int i = lane; i < n_v; i += 64) {
    ymax = fmax(ymax, y[i]);
    if (y[i] < ymin) {
      ymin = y[i];
      kmin = i;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    ymax = fmax(ymax, __shfl_xor(ymax, off, 64));
    const double om = __shfl_xor(ymin, off, 64);
    const int ok = __shfl_xor(kmin, off, 64);
    if (om < ymin || (om == ymin && ok < kmin)) {
      ymin = om;
      kmin = ok;
    }
  }
  const double c0 = ymax;
  const double a0 = c0 - ymin;
  const double half = c0 - 0.5 * a0;
  int first = n_v, last = -1;
  for (int i = lane; i < n_v; i += 64) {
    if (y[i] <= half) {
      first = min(first, i);
      last = max(last, i);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    first = min(first, __shfl_xor(first, off, 64));
    last = max(last, __shfl_xor(last, off, 64));
  }
  const double width = (last > first) ? dv * (last - first) : dv;
  double p[4] = {c0, a0, v0 + dv * kmin, fmax(width, dv) / FWHM_PER_SIGMA};

  soap_rv res;
  res.status = 0;
  if (!(a0 > 0.0) || !isfinite(c0) || !isfinite(ymin)) {
    res.status = 2;
    res.iters = 0;
  } else {
    double chi2, jtj[10], jtr[4];
    gf_eval(y, n_v, v0, dv, p, true, chi2, jtj, jtr);
    double lam = 1e-3;
    int it = 0;
    res.status = 1;
    for (; it < 200; ++it) {
      bool accepted = false;
      double step[4] = {0, 0, 0, 0};
      double chi2n = chi2;
      while (lam < 1e20) {
        double x[4];
        if (gf_solve(jtj, jtr, lam, x)) {
          double pn[4] = {p[0] + x[0], p[1] + x[1], p[2] + x[2], p[3] + x[3]};
          double dummy10[10], dummy4[4];
          gf_eval(y, n_v, v0, dv, pn, false, chi2n, dummy10, dummy4);
          if (chi2n <= chi2) {
            for (int q = 0; q < 4; ++q) {
              step[q] = x[q];
              p[q] = pn[q];
            }
            accepted = true;
            lam = fmax(lam * 0.1, 1e-12);
            break;
          }
        }
        lam *= 10.0;
      }
      if (!accepted) {
        // no downhill step at any damping: at the minimum to rounding
        res.status = 0;
        break;
      }
      const double dchi = chi2 - chi2n;
      chi2 = chi2n;
      gf_eval(y, n_v, v0, dv, p, true, chi2, jtj, jtr);
      if (fabs(step[2]) < 1e-11 && fabs(step[3]) < 1e-11 * fabs(p[3]) && dchi <= 1e-14 * chi2 + 1e-300) {
        res.status = 0;
        ++it;
        break;
      }
    }
    res.iters = it;
    res.chi2 = chi2;
  }
  res.rv_kms = p[2];
  res.sigma_kms = fabs(p[3]);
  res.fwhm_kms = FWHM_PER_SIGMA * fabs(p[3]);
  res.c0 = p[0];
  res.amp = p[1];
  if (res.status == 2) res.chi2 = 0.0;
  if (lane == 0) out[s] = res;
}

hipError_t launch_ccf(soap_ctx* c, const void* d_flux, int64_t n_spec, const double* d_mask, int n_lines,
                      double* d_part, double* d_ccf) {
  const int nlb = ccf_line_blocks(n_lines);
  dim3 grid(nlb, (unsigned)((n_spec + CCF_SB - 1) / CCF_SB));
  if (c->prec == SOAP_PREC_FP32)
    hipLaunchKernelGGL(k_ccf<float>, grid, dim3(CCF_THREADS), 0, c->stream, c->P, n_spec,
                       (const float*)d_flux, n_lines, (const double2*)d_mask, c->mask_nv, c->mask_v0,
                       c->mask_dv, c->mask_h, c->dln, d_part);
  else
    hipLaunchKernelGGL(k_ccf<double>, grid, dim3(CCF_THREADS), 0, c->stream, c->P, n_spec,
                       (const double*)d_flux, n_lines, (const double2*)d_mask, c->mask_nv, c->mask_v0,
                       c->mask_dv, c->mask_h, c->dln, d_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nt = n_spec * c->mask_nv;
  hipLaunchKernelGGL(k_ccf_reduce, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, c->stream, nlb, n_spec,
                     c->mask_nv, d_part, d_ccf);
  return hipGetLastError();
}

hipError_t launch_mask_prep(soap_ctx* c, const double* d_lnl, const double* d_w, int n, double* d_mask) {
  hipLaunchKernelGGL(k_mask_prep, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, c->ln0, c->dln, d_lnl, d_w,
                     (double2*)d_mask);
  return hipGetLastError();
}

hipError_t launch_gfit(soap_ctx* c, const double* d_ccf, int64_t n_spec, soap_rv* d_rv) {
  hipLaunchKernelGGL(k_gfit, dim3((unsigned)n_spec), dim3(64), 0, c->stream, n_spec, c->mask_nv, c->mask_v0,
                     c->mask_dv, d_ccf, d_rv);
  return hipGetLastError();
}

}  // namespace soap
