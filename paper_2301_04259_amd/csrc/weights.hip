// Per-phase active-region weights (section 3.3, Algorithm 5).
//
// For each phase one workgroup
//   1. rotates every region centre to the phase (longitude + 360 deg * phase,
//      axis tilted by the inclination) and takes the bounding box of the
//      visible caps;
//   2. walks the disk columns of that box, one wave64 per column and one lane
//      per cell: a cell belongs to a region when the angle between its surface
//      point and the centre is at most asin(radius); the InfoMap owner is the
//      last region in list order that covers it;
//   3. sums, per column, the weights A I(mu) of active cells per mu bin: the
//      quiet removal (-A I, every active cell) and the active terms
//      (+A I c, per region type; c = the region's scalar contrast in the
//      scalar mode of Eqs. 1 and 3, 1 otherwise).  Each lane accumulates its
//      cells (FP32 + Kahan in the FP32 mode, FP64 otherwise), the 64 lane
//      partials are reduced in FP64;
//   4. collapses the column sums onto the integer offsets of the column's
//      shift (weights 1 - w at j = c, w at j = c - 1, Eq. 11) in FP64, in a
//      per-wave table, and finally sums the waves in a fixed order.
// The result is a dense tap table K[phase][g][j] with g = type * B + bin
// (type 0 = quiet removal, 1 = spot, 2 = facula) and j - jmin in [0, J).
//
// k_compact then turns the taps of each chunk of phases into the list the
// apply kernel walks: virtual groups (a group and a window of APPLY_JW
// offsets) and, per phase, runs of <= 4 consecutive taps.
#include "soap_internal.hpp"

namespace soap {

namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ unsigned long long wor(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off, 64);
  return v;
}

constexpr int MAXC = 4;  // cells cached per lane per row pass (256 rows)

}  // namespace

template <bool KAHAN32>
__global__ void __launch_bounds__(1024) k_weights(int N, int B, int J, int jmin, double u1, double u2,
                                                  double incl, int effect, int cmode,
                                                  const double* __restrict__ mu_b,
                                                  const int* __restrict__ col_c,
                                                  const double* __restrict__ col_w,
                                                  const Region* __restrict__ reg, int n_reg,
                                                  const double* __restrict__ phases,
                                                  double* __restrict__ K) {
  extern __shared__ double lds[];
  __shared__ double rcx[MAX_REGIONS], rcy[MAX_REGIONS], rcz[MAX_REGIONS], rcos[MAX_REGIONS],
      rscal[MAX_REGIONS];
  __shared__ int rtype[MAX_REGIONS];
  __shared__ int box[4];

  const int ph = blockIdx.x;
  const int nw = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int G = 3 * B;
  const int GJ = G * J;
  const double phase = phases[ph];
  const double area = (2.0 / N) * (2.0 / N);

  for (int t = threadIdx.x; t < nw * GJ; t += blockDim.x) lds[t] = 0.0;
  if (threadIdx.x < n_reg) {
    const Region r = reg[threadIdx.x];
    double cx, cy, cz;
    region_centre(r.lat_deg, r.lon_deg, phase, incl, &cx, &cy, &cz);
    rcx[threadIdx.x] = cx;
    rcy[threadIdx.x] = cy;
    rcz[threadIdx.x] = cz;
    {
#pragma clang fp contract(off)
      rcos[threadIdx.x] = sqrt(1.0 - r.radius * r.radius);
    }
    rtype[threadIdx.x] = r.type;
    rscal[threadIdx.x] = (cmode == SOAP_CONTRAST_SCALAR && effect != SOAP_EFFECT_BCONV) ? r.contrast : 1.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // bounding box of the caps that reach the visible hemisphere; a cap
    // point p satisfies |p - c| <= 2 sin(alpha / 2) = sqrt(2 - 2 cos alpha),
    // which bounds its projected distance from the centre
    double xlo = 2.0, xhi = -2.0, ylo = 2.0, yhi = -2.0;
    for (int r = 0; r < n_reg; ++r) {
      double rad = sqrt(1.0 - rcos[r] * rcos[r]);
      if (rcz[r] <= -rad - 1e-12) continue;
      double d = sqrt(fmax(0.0, 2.0 - 2.0 * rcos[r])) + 1e-9;
      xlo = fmin(xlo, rcx[r] - d);
      xhi = fmax(xhi, rcx[r] + d);
      ylo = fmin(ylo, rcy[r] - d);
      yhi = fmax(yhi, rcy[r] + d);
    }
    int i0 = (int)floor((xlo + 1.0) * 0.5 * N) - 1;
    int i1 = (int)ceil((xhi + 1.0) * 0.5 * N) + 1;
    int k0 = (int)floor((ylo + 1.0) * 0.5 * N) - 1;
    int k1 = (int)ceil((yhi + 1.0) * 0.5 * N) + 1;
    box[0] = max(i0, 0);
    box[1] = min(i1, N - 1);
    box[2] = max(k0, 0);
    box[3] = min(k1, N - 1);
  }
  __syncthreads();
  const int i0 = box[0], i1 = box[1], k0 = box[2], k1 = box[3];
  double* myK = lds + wave * GJ;

  for (int i = i0 + wave; i <= i1; i += nw) {
    const double x = cell_coord(i, N);
    const int ci = col_c[i];
    const double wi = col_w[i];
    for (int kbase = k0; kbase <= k1; kbase += 64 * MAXC) {
      int cb[MAXC];      // bin | (type << 8), or -1 when not active
      double cw[MAXC];   // A I(mu)
      double cs[MAXC];   // owner contrast scale
      unsigned long long m1 = 0, m2 = 0;
#pragma unroll
      for (int q = 0; q < MAXC; ++q) {
        cb[q] = -1;
        cw[q] = 0.0;
        cs[q] = 0.0;
        const int k = kbase + lane + 64 * q;
        if (k <= k1) {
          const double y = cell_coord(k, N);
          double r2;
          {
#pragma clang fp contract(off)
            r2 = x * x + y * y;
          }
          if (r2 < 1.0) {
            const double mu = sqrt(1.0 - r2);
            int own = -1;
            for (int r = 0; r < n_reg; ++r) {
              double dot;
              {
#pragma clang fp contract(off)
                dot = x * rcx[r] + y * rcy[r] + mu * rcz[r];
              }
              if (dot >= rcos[r]) own = r;
            }
            if (own >= 0) {
              const int b = nearest_bin(mu, mu_b, B);
              const int t = rtype[own];
              cb[q] = b | (t << 8);
              cw[q] = area * limb_dark(mu, u1, u2);
              cs[q] = rscal[own];
              if (t == SOAP_SPOT) m1 |= 1ull << b;
              else m2 |= 1ull << b;
            }
          }
        }
      }
      m1 = wor(m1);
      m2 = wor(m2);
      unsigned long long mall = m1 | m2;
      while (mall) {
        const int b = __builtin_ctzll(mall);
        mall &= mall - 1;
        double prem, pspot, pfac;
        if (KAHAN32) {
          float s0 = 0.f, c0 = 0.f, s1 = 0.f, c1 = 0.f, s2 = 0.f, c2 = 0.f;
#pragma unroll
          for (int q = 0; q < MAXC; ++q) {
            if (cb[q] >= 0 && (cb[q] & 0xff) == b) {
              const float v = (float)cw[q];
              const float va = (float)(cw[q] * cs[q]);
              float yk = v - c0, t = s0 + yk;
              c0 = (t - s0) - yk;
              s0 = t;
              if ((cb[q] >> 8) == SOAP_SPOT) {
                yk = va - c1;
                t = s1 + yk;
                c1 = (t - s1) - yk;
                s1 = t;
              } else {
                yk = va - c2;
                t = s2 + yk;
                c2 = (t - s2) - yk;
                s2 = t;
              }
            }
          }
          prem = (double)s0 - (double)c0;
          pspot = (double)s1 - (double)c1;
          pfac = (double)s2 - (double)c2;
        } else {
          double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
          for (int q = 0; q < MAXC; ++q) {
            if (cb[q] >= 0 && (cb[q] & 0xff) == b) {
              s0 += cw[q];
              if ((cb[q] >> 8) == SOAP_SPOT) s1 += cw[q] * cs[q];
              else s2 += cw[q] * cs[q];
            }
          }
          prem = s0;
          pspot = s1;
          pfac = s2;
        }
        const double Wrem = wsum(prem);
        const double Wspot = (m1 >> b) & 1 ? wsum(pspot) : 0.0;
        const double Wfac = (m2 >> b) & 1 ? wsum(pfac) : 0.0;
        const int ja = ci - jmin, jb = ci - 1 - jmin;
        if (lane == 0 && jb >= 0 && ja < J) {
          double* kr = myK + (0 * B + b) * J;
          kr[ja] -= (1.0 - wi) * Wrem;
          kr[jb] -= wi * Wrem;
          if (Wspot != 0.0) {
            kr = myK + (SOAP_SPOT * B + b) * J;
            kr[ja] += (1.0 - wi) * Wspot;
            kr[jb] += wi * Wspot;
          }
          if (Wfac != 0.0) {
            kr = myK + (SOAP_FACULA * B + b) * J;
            kr[ja] += (1.0 - wi) * Wfac;
            kr[jb] += wi * Wfac;
          }
        }
      }
    }
  }
  __syncthreads();
  double* out = K + (int64_t)ph * GJ;
  for (int t = threadIdx.x; t < GJ; t += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[w * GJ + t];
    out[t] = s;
  }
}

// one block per chunk of APPLY_PC phases
template <typename T>
__global__ void __launch_bounds__(256) k_compact(int n_ph, int G, int J, int jmin, const double* __restrict__ K,
                                                 VGroup* __restrict__ vgs, int* __restrict__ nvg,
                                                 Entry<T>* __restrict__ ents, int vg_cap, int ent_cap) {
  extern __shared__ int sm[];
  int* s_cnt = sm;             // [G] virtual groups per group
  int* s_base = sm + G;        // [G]
  int* s_ecnt = sm + 2 * G;    // [vg_cap] entries per virtual group
  int* s_ebase = s_ecnt + vg_cap;
  const int chunk = blockIdx.x;
  const int p0 = chunk * APPLY_PC;
  const int np = min(APPLY_PC, n_ph - p0);
  const int GJ = G * J;
  const double* Kc = K + (int64_t)p0 * GJ;
  VGroup* vg = vgs + (int64_t)chunk * vg_cap;
  Entry<T>* en = ents + (int64_t)chunk * ent_cap;
  const int nwin_max = (J + APPLY_JW - 1) / APPLY_JW;

  // pass 1: windows with any tap per group
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    unsigned long long any = 0;
    for (int p = 0; p < np; ++p)
      for (int j = 0; j < J; ++j)
        if (Kc[(int64_t)p * GJ + g * J + j] != 0.0) any |= 1ull << j;
    int cnt = 0;
    if (any) {
      const int lo = __builtin_ctzll(any);
      for (int wv = 0; wv < nwin_max; ++wv) {
        const int a = lo + wv * APPLY_JW;
        if (a >= J) break;
        const unsigned long long wm = (any >> a) & ((1ull << APPLY_JW) - 1);
        if (wm) ++cnt;
      }
    }
    s_cnt[g] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int g = 0; g < G; ++g) {
      s_base[g] = acc;
      acc += s_cnt[g];
    }
    nvg[chunk] = acc;
  }
  __syncthreads();
  // pass 2: virtual group records and entry counts
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    if (!s_cnt[g]) continue;
    unsigned long long any = 0;
    for (int p = 0; p < np; ++p)
      for (int j = 0; j < J; ++j)
        if (Kc[(int64_t)p * GJ + g * J + j] != 0.0) any |= 1ull << j;
    const int lo = __builtin_ctzll(any);
    int v = s_base[g];
    for (int wv = 0; wv < nwin_max; ++wv) {
      const int a = lo + wv * APPLY_JW;
      if (a >= J) break;
      if (!((any >> a) & ((1ull << APPLY_JW) - 1))) continue;
      int ecount = 0;
      for (int p = 0; p < np; ++p) {
        const double* kr = Kc + (int64_t)p * GJ + g * J;
        int q = 0;
        while (q < APPLY_JW) {
          if (a + q < J && kr[a + q] != 0.0) {
            ++ecount;
            q += 4;
          } else {
            ++q;
          }
        }
      }
      vg[v].g = g;
      vg[v].jlo = jmin + a;
      s_ecnt[v] = ecount;
      ++v;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    const int n = nvg[chunk];
    for (int v = 0; v < n; ++v) {
      s_ebase[v] = acc;
      acc += s_ecnt[v];
    }
  }
  __syncthreads();
  // pass 3: entries, phase-major inside each virtual group
  const int n = nvg[chunk];
  for (int v = threadIdx.x; v < n; v += blockDim.x) {
    const int g = vg[v].g;
    const int a = vg[v].jlo - jmin;
    int e = s_ebase[v];
    for (int p = 0; p < APPLY_PC; ++p) {
      vg[v].off[p] = e;
      if (p >= np) continue;
      const double* kr = Kc + (int64_t)p * GJ + g * J;
      int q = 0;
      while (q < APPLY_JW) {
        if (a + q < J && kr[a + q] != 0.0) {
          int w = 1;
          for (int t = 1; t < 4 && q + t < APPLY_JW && a + q + t < J; ++t)
            if (kr[a + q + t] != 0.0) w = t + 1;
          Entry<T> E;
          E.code = q * 4 + (w - 1);
          E.pad = 0;
          for (int t = 0; t < 4; ++t) E.k[t] = (t < w) ? (T)kr[a + q + t] : (T)0;
          en[e++] = E;
          q += 4;
        } else {
          ++q;
        }
      }
    }
    vg[v].off[APPLY_PC] = e;
  }
}

hipError_t launch_weights(soap_ctx* c, const Region* d_reg, int n_reg, const double* d_ph, int n_ph,
                          int effect, double* d_K) {
  const int G = 3 * c->B;
  const size_t per_wave = (size_t)G * c->J * sizeof(double);
  // dynamic LDS stays below 60 KB so that with the static arrays the block
  // fits a 64 KB workgroup allocation
  int nw = (int)std::min<size_t>(16, (60 * 1024) / per_wave);
  if (nw < 1) nw = 1;
  const size_t lds = nw * per_wave;
  if (c->prec == SOAP_PREC_FP32)
    hipLaunchKernelGGL(k_weights<true>, dim3(n_ph), dim3(64 * nw), lds, c->stream, c->N, c->B, c->J, c->jmin,
                       c->u1, c->u2, c->incl, effect, c->cmode, c->d_mu, c->d_col_c, c->d_col_w, d_reg, n_reg,
                       d_ph, d_K);
  else
    hipLaunchKernelGGL(k_weights<false>, dim3(n_ph), dim3(64 * nw), lds, c->stream, c->N, c->B, c->J,
                       c->jmin, c->u1, c->u2, c->incl, effect, c->cmode, c->d_mu, c->d_col_c, c->d_col_w,
                       d_reg, n_reg, d_ph, d_K);
  return hipGetLastError();
}

hipError_t launch_compact(soap_ctx* c, const double* d_K, int n_ph, VGroup* d_vg, int* d_nvg, void* d_ent,
                          int vg_cap, int ent_cap) {
  const int G = 3 * c->B;
  const int n_chunks = (n_ph + APPLY_PC - 1) / APPLY_PC;
  const size_t lds = (size_t)(2 * G + 2 * vg_cap) * sizeof(int);
  if (c->prec == SOAP_PREC_FP32)
    hipLaunchKernelGGL(k_compact<float>, dim3(n_chunks), dim3(256), lds, c->stream, n_ph, G, c->J, c->jmin, d_K,
                       d_vg, d_nvg, (Entry<float>*)d_ent, vg_cap, ent_cap);
  else
    hipLaunchKernelGGL(k_compact<double>, dim3(n_chunks), dim3(256), lds, c->stream, n_ph, G, c->J, c->jmin,
                       d_K, d_vg, d_nvg, (Entry<double>*)d_ent, vg_cap, ent_cap);
  return hipGetLastError();
}

}  // namespace soap
