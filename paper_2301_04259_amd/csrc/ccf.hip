// CCF against a line mask and Gaussian fit of the CCF (section 4.1: RVs from
// cross-correlation with a line mask and the mean of a fitted Gaussian).
//
// CCF: pixel m is a constant-flux bin [m, m+1) in the pixel coordinate
// q = (ln(lambda) - ln0)/dln + 1/2.  Mask line l sits at u_l in that
// coordinate; at trial velocity v_k its hole spans [u_l + a_k^-, u_l + a_k^+]
// with a_k^+- = atanh((v_k +- h)/c)/dln (the ln of the Eq. 6 factor).
// CCF_k = sum_l w_l sum_m F_m * overlap(bin m, hole), existing pixels only.
// The line positions, the hole edges per velocity and the split of the mask
// into blocks of lines and batches of nearby lines are built on the host
// once per mask.  Layout: one block per (block of lines, block of SB
// spectra), one thread per velocity; each thread keeps SB double
// accumulators and reuses its hole geometry for every spectrum of the block.
// Partial sums per line block are added in a fixed order by the fit kernel,
// so results repeat bit for bit.
//
// Fit: one wave64 per CCF; damped Newton (Levenberg-Marquardt damping) in
// double on the unweighted least squares of c0 - a exp(-(v - mu)^2 /
// (2 sigma^2)); the gradient, J^T J and the second-derivative sums are wave
// reductions, the 4 x 4 damped system is solved by Cholesky in every lane.
// Start values: c0 = max, a = c0 - min, mu at the vertex of the parabola
// through the minimum and its neighbours, sigma from the half-depth width
// with the crossings interpolated between samples.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "soap_internal.hpp"
#include "wave.hpp"

namespace soap {

constexpr int CCF_LB = 32;        // mask lines per block (one partial CCF row each)
constexpr int CCF_SB = 8;         // spectra per block
constexpr int CCF_THREADS = 192;  // one thread per velocity (A velocities each past 192)
constexpr int CCF_STG_MAX = 512;  // widest staged span of a batch, in pixels
// a line's hole centre, in pixels, is kept within this margin of the grid:
// lines further out reach no pixel
constexpr double CCF_U_MARGIN = 4096.0;

int ccf_line_blocks(int n_lines) { return (n_lines + CCF_LB - 1) / CCF_LB; }
int ccf_span_pixels(bool) { return CCF_STG_MAX; }

namespace {

// 4 consecutive elements of 16-byte-aligned memory in their own type
template <typename T>
__device__ __forceinline__ void get4t(T* x, const T* p) {
  if constexpr (sizeof(T) == 4) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
  } else {
    const double2 a = reinterpret_cast<const double2*>(p)[0];
    const double2 b = reinterpret_cast<const double2*>(p)[1];
    x[0] = a.x;
    x[1] = a.y;
    x[2] = b.x;
    x[3] = b.y;
  }
}

}  // namespace

// One block per (CCF_LB mask lines, CCF_SB spectra).  The block walks the
// batches of its lines (host-built: consecutive lines whose holes, at every
// trial velocity, stay inside a span of STG pixels).  A batch's span of the
// block's spectra is staged pixel-major in LDS, [pixel][spectrum], so that
// one thread reads the SB values of a pixel with 16-byte loads; two stage
// buffers alternate, the next batch's loads are in flight while one is
// used, and one barrier per batch separates them.  Pixels outside the
// spectrum are staged as zeros.  Each thread computes its holes' pixel
// overlaps once per line (in double: the hole edges come from differences of
// nearby pixel coordinates) and applies them to every staged spectrum with
// FMAs in the flux precision: a block's partial CCF sums at most 32 lines x
// a few pixels in FP32 for float spectra, and the partials of the line blocks
// are added in double by the fit kernel.
// Line block lb, spectrum block sb.
template <typename T, int A, int NPX, int STG>
__device__ __forceinline__ void ccf_block(int P, int64_t n_spec, const T* __restrict__ F,
                                          const double2* __restrict__ lines, const double2* __restrict__ edges,
                                          const int4* __restrict__ batches, const int* __restrict__ bfirst,
                                          int n_v, T* __restrict__ part, int lb, int sb) {
  constexpr int SB = CCF_SB;
  constexpr int R = (STG + CCF_THREADS - 1) / CCF_THREADS;  // staged pixels per thread
  static_assert(SB % 4 == 0, "16-byte stage rows");
  __shared__ __align__(16) T st[2][STG][SB];
  __shared__ double2 s_line[CCF_LB];
  __shared__ double2 s_ed[A * CCF_THREADS];
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)sb * SB;
  const int ns = (int)min<int64_t>(SB, n_spec - s0);
  const int b0 = bfirst[lb], b1 = bfirst[lb + 1];
  const int l0 = batches[b0].y;
  const int nl = batches[b1 - 1].z - l0;
  if (tid < nl) s_line[tid] = lines[l0 + tid];
  // lanes past the velocity grid repeat its last velocity (results dropped);
  // the edges go through LDS so that no global load is pending in the loop
#pragma unroll
  for (int a = 0; a < A; ++a) s_ed[tid + a * CCF_THREADS] = edges[min(tid + a * CCF_THREADS, n_v - 1)];
  __syncthreads();
  double alo[A], ahi[A];
  T acc[A][SB];
#pragma unroll
  for (int a = 0; a < A; ++a) {
    const double2 e = s_ed[tid + a * CCF_THREADS];
    alo[a] = e.x;
    ahi[a] = e.y;
#pragma unroll
    for (int s = 0; s < SB; ++s) acc[a][s] = T(0);
  }
  T vals[R][SB];
  // only the batch's read span (batches[bi].w <= STG pixels) is loaded and
  // staged: no hole of the batch reads past it
  auto load = [&](int bi) {
    if (bi >= b1) return;
    const int lo = batches[bi].x, span = batches[bi].w;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (tid + r * CCF_THREADS < span) {
        const int m = min(max(lo + tid + r * CCF_THREADS, 0), P - 1);
#pragma unroll
        for (int s = 0; s < SB; ++s) vals[r][s] = F[(s0 + min(s, ns - 1)) * (int64_t)P + m];
      }
    }
  };
  auto put = [&](int bi) {
    if (bi >= b1) return;
    const int lo = batches[bi].x, span = batches[bi].w;
    T(*sb)[SB] = st[(bi - b0) & 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + r * CCF_THREADS;
      if (i < span) {
        const int m = lo + i;
        const bool ok = m >= 0 && m < P;
#pragma unroll
        for (int s = 0; s < SB; ++s) sb[i][s] = ok ? vals[r][s] : T(0);
      }
    }
  };
  load(b0);
  put(b0);
  load(b0 + 1);
  __syncthreads();
  for (int bi = b0; bi < b1; ++bi) {
    const int4 B = batches[bi];
    const T(*sb)[SB] = st[(bi - b0) & 1];
    for (int l = B.y; l < B.z; ++l) {
      const double2 mw = s_line[l - l0];
#pragma unroll
      for (int a = 0; a < A; ++a) {
        const double qlo = mw.x + alo[a];
        const double qhi = mw.x + ahi[a];
        const double fa = floor(qlo);
        const int i0 = (int)fa - B.x;
        double w[NPX];
        if constexpr (NPX == 2) {
          // a hole narrower than a pixel: the first pixel takes the part of
          // the hole below fa + 1, the second the rest
          const double e1 = fa + 1.0;
          w[0] = mw.y * (fmin(qhi, e1) - qlo);
          w[1] = mw.y * fmax(qhi - e1, 0.0);
        } else {
          // pixel px covers [fa + px, fa + px + 1); the first pixel's lower
          // edge is the hole's, pixels past the hole get weight zero
#pragma unroll
          for (int px = 0; px < NPX; ++px) {
            const double mlo = fa + (double)px;
            w[px] = mw.y * fmax(fmin(qhi, mlo + 1.0) - (px == 0 ? qlo : mlo), 0.0);
          }
        }
#pragma unroll
        for (int px = 0; px < NPX; ++px) {
          T f[SB];
#pragma unroll
          for (int c = 0; c < SB / 4; ++c) get4t(&f[4 * c], &sb[i0 + px][4 * c]);
          const T wp = (T)w[px];
#pragma unroll
          for (int s = 0; s < SB; ++s) acc[a][s] = fma(wp, f[s], acc[a][s]);
        }
      }
    }
    put(bi + 1);
    load(bi + 2);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < A; ++a) {
    const int k = tid + a * CCF_THREADS;
    if (k >= n_v) break;
#pragma unroll
    for (int s = 0; s < SB; ++s)
      if (s < ns) part[((int64_t)lb * n_spec + s0 + s) * n_v + k] = acc[a][s];
  }
}

template <typename T, int A, int NPX, int STG>
__global__ void __launch_bounds__(CCF_THREADS) k_ccf(int P, int64_t n_spec, const T* __restrict__ F,
                                                     const double2* __restrict__ lines,
                                                     const double2* __restrict__ edges,
                                                     const int4* __restrict__ batches,
                                                     const int* __restrict__ bfirst, int n_v,
                                                     T* __restrict__ part) {
  ccf_block<T, A, NPX, STG>(P, n_spec, F, lines, edges, batches, bfirst, n_v, part, blockIdx.x, blockIdx.y);
}

// Work-list form over many spectra sets with one mask layout: blk[b] =
// (set, line block, spectrum block).
template <typename T, int A, int NPX, int STG>
__global__ void __launch_bounds__(CCF_THREADS) k_ccf_batch(const CcfBatchSet* __restrict__ sets,
                                                           const int4* __restrict__ blk, int n_v) {
  const int4 t = blk[blockIdx.x];
  const CcfBatchSet c = sets[t.x];
  const unsigned char* tb = c.tables;
  ccf_block<T, A, NPX, STG>(c.P, c.n_spec, static_cast<const T*>(c.flux), reinterpret_cast<const double2*>(tb),
                            reinterpret_cast<const double2*>(tb + c.off_edges),
                            reinterpret_cast<const int4*>(tb + c.off_batch),
                            reinterpret_cast<const int*>(tb + c.off_bfirst), n_v, static_cast<T*>(c.part), t.y, t.z);
}

// Host tables of one mask (section 4.1's CCF with the holes of Eq. 6),
// appended to blob with 16-byte-aligned sections: lines (u, w) double2[nl],
// hole edges (a^-, a^+) double2[n_v], batches int4 {first staged pixel,
// first line, end line, pixels read}, and per line block the index of its first batch
// (int[n_lb + 1]).  Batches hold consecutive lines whose reads, from the
// floor of the lowest hole edge to NPX pixels past the floor of the highest,
// fit a span of STG pixels.
bool ccf_build_tables(soap_ctx* c, const double* lnl, const double* wl, int nl, std::vector<unsigned char>& blob,
                      std::string& err) {
  const int nv = c->mask_nv;
  std::vector<double2> ln(nl), ed(nv);
  for (int l = 0; l < nl; ++l) {
    const double u = (lnl[l] - c->ln0) / c->dln + 0.5;
    ln[l] = make_double2(std::fmin(std::fmax(u, -CCF_U_MARGIN), (double)c->P + CCF_U_MARGIN), wl[l]);
  }
  double wmax = 0.0;
  for (int k = 0; k < nv; ++k) {
    const double vk = c->mask_v0 + c->mask_dv * k;
    ed[k] = make_double2(std::atanh((vk - c->mask_h) / C_KMS) / c->dln, std::atanh((vk + c->mask_h) / C_KMS) / c->dln);
    wmax = std::fmax(wmax, ed[k].y - ed[k].x);
  }
  const int npx = wmax < 1.0 ? 2 : (wmax < 2.0 ? 3 : (wmax < 4.0 ? 5 : 10));
  // the edges grow with k (atanh is increasing), so these bound every hole
  const double amin = ed[0].x, amax = ed[nv - 1].y;
  auto span_lo = [&](int l) { return (int)std::floor(ln[l].x + amin); };
  auto span_end = [&](int l) { return (int)std::floor(ln[l].x + amax) + npx; };
  // lines whose reads all fall outside the spectrum add exactly zero to
  // every velocity (their staged pixels are zeros): they are left out of the
  // tables (one is kept when none reaches the spectrum, so that there is a
  // line block)
  {
    int kept = 0;
    for (int l = 0; l < nl; ++l)
      if (span_end(l) > 0 && span_lo(l) < (int64_t)c->P) ln[kept++] = ln[l];
    if (kept == 0) kept = 1;
    nl = kept;
    ln.resize(nl);
  }
  c->ccf_nl = nl;
  int widest = 0;
  for (int l = 0; l < nl; ++l) widest = std::max(widest, span_end(l) - span_lo(l));
  if (widest > CCF_STG_MAX) {
    err = "the velocity grid and holes span " + std::to_string(widest) + " pixels, beyond the supported " +
          std::to_string(CCF_STG_MAX);
    return false;
  }
  const int stg = widest <= 256 ? 256 : CCF_STG_MAX;
  const int nlb = ccf_line_blocks(nl);
  std::vector<int4> bat;
  std::vector<int> bfirst(nlb + 1);
  for (int b = 0; b < nlb; ++b) {
    bfirst[b] = (int)bat.size();
    const int l0 = b * CCF_LB, l1 = std::min(nl, l0 + CCF_LB);
    int lo = span_lo(l0), hi = span_end(l0), beg = l0;
    for (int l = l0 + 1; l < l1; ++l) {
      const int nlo = std::min(lo, span_lo(l)), nhi = std::max(hi, span_end(l));
      if (nhi - nlo > stg) {
        bat.push_back(make_int4(lo, beg, l, hi - lo));
        lo = span_lo(l);
        hi = span_end(l);
        beg = l;
      } else {
        lo = nlo;
        hi = nhi;
      }
    }
    bat.push_back(make_int4(lo, beg, l1, hi - lo));
  }
  bfirst[nlb] = (int)bat.size();
  auto al16 = [](size_t v) { return (v + 15) & ~size_t(15); };
  const size_t o_ed = al16(sizeof(double2) * nl);
  const size_t o_bat = al16(o_ed + sizeof(double2) * nv);
  const size_t o_bf = al16(o_bat + sizeof(int4) * bat.size());
  blob.assign(al16(o_bf + sizeof(int) * bfirst.size()), 0);
  std::memcpy(blob.data(), ln.data(), sizeof(double2) * nl);
  std::memcpy(blob.data() + o_ed, ed.data(), sizeof(double2) * nv);
  std::memcpy(blob.data() + o_bat, bat.data(), sizeof(int4) * bat.size());
  std::memcpy(blob.data() + o_bf, bfirst.data(), sizeof(int) * bfirst.size());
  c->ccf_off_edges = o_ed;
  c->ccf_off_batch = o_bat;
  c->ccf_off_bfirst = o_bf;
  c->ccf_nbatch = (int)bat.size();
  c->ccf_npx = npx;
  c->ccf_stg = stg;
  c->mask_hole_px = wmax;
  return true;
}

namespace {

constexpr double FWHM_PER_SIGMA = 2.3548200450309493;  // 2 sqrt(2 ln 2)
constexpr int CCF_FIN_THREADS = 256;
constexpr int64_t CCF_FIT_WAVES_FROM = 512;  // spectra per call above which one wave fits each

// Sums of the fit at p, identical in every lane: S[0] = chi^2,
// S[1..4] = g = J^T r, S[5..14] = J^T J (upper triangle, row by row),
// S[15..19] = sum r d2f/dp_a dp_b for (amp, mu), (amp, sigma), (mu, mu),
// (mu, sigma), (sigma, sigma) (the only second derivatives that are not
// zero), with f = c0 - amp e, e = exp(-(v - mu)^2 / (2 sigma^2)), r = f - y
// and parameters ordered (c0, amp, mu, sigma).
template <int NPT>
__device__ void gf_eval(const double (&y)[NPT], int n_v, double v0, double dv, const double p[4],
                        double S[20]) {
  const int lane = threadIdx.x & 63;
  double v[16], w[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = w[q] = 0.0;
  const double is = 1.0 / p[3];
  const double is2 = is * is;
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    if (64 * t >= n_v) break;  // uniform
    const int i = lane + 64 * t;
    if (i < n_v) {
      const double x = v0 + dv * i;
      const double d = x - p[2];
      const double z = d * d * is2;  // (d / sigma)^2
      const double e = exp(-0.5 * z);
      const double ae = p[1] * e;
      const double r = p[0] - ae - y[t];
      const double g[4] = {1.0, -e, -ae * d * is2, -ae * z * is};
      v[0] += r * r;
#pragma unroll
      for (int r0 = 0; r0 < 4; ++r0) v[1 + r0] += g[r0] * r;
      int q = 5;
#pragma unroll
      for (int r0 = 0; r0 < 4; ++r0)
#pragma unroll
        for (int r1 = r0; r1 < 4; ++r1) v[q++] += g[r0] * g[r1];
      const double re = r * e;
      w[0] += re * (-d * is2);                       // (amp, mu)
      w[1] += re * (-z * is);                        // (amp, sigma)
      w[2] += r * (-ae * (z - 1.0) * is2);           // (mu, mu)
      w[3] += r * (-ae * d * (z - 2.0) * is2 * is);  // (mu, sigma)
      w[4] += r * (-ae * z * (z - 3.0) * is2);       // (sigma, sigma)
    }
  }
  const double tv = butterfly16_rows(v, lane);
  const double tw = butterfly16_rows(w, lane);
#pragma unroll
  for (int q = 0; q < 15; ++q) S[q] = read_lane(tv, q);
#pragma unroll
  for (int q = 0; q < 5; ++q) S[15 + q] = read_lane(tw, q);
}

// Solves (H + lam diag(J^T J)) x = -g by Cholesky, H = J^T J (+ the
// second-derivative sums when newton is set).  False when the matrix is not
// positive definite.
__device__ bool gf_solve(const double S[20], bool newton, double lam, double x[4]) {
  double A[4][4];
  int q = 5;
  for (int r0 = 0; r0 < 4; ++r0)
    for (int r1 = r0; r1 < 4; ++r1) {
      A[r0][r1] = S[q];
      A[r1][r0] = S[q];
      ++q;
    }
  if (newton) {
    A[1][2] += S[15];
    A[2][1] += S[15];
    A[1][3] += S[16];
    A[3][1] += S[16];
    A[2][2] += S[17];
    A[2][3] += S[18];
    A[3][2] += S[18];
    A[3][3] += S[19];
  }
  const double dg[4] = {S[5], S[9], S[12], S[14]};  // diag(J^T J)
  for (int r = 0; r < 4; ++r) A[r][r] += lam * dg[r];
  double L[4][4] = {{0}}, rd[4];
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[i][i] = sqrt(s);
        rd[i] = 1.0 / L[i][i];
      } else {
        L[i][j] = s * rd[j];
      }
    }
  }
  double z[4];
  for (int i = 0; i < 4; ++i) {
    double s = -S[1 + i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * z[k];
    z[i] = s * rd[i];
  }
  for (int i = 3; i >= 0; --i) {
    double s = z[i];
    for (int k = i + 1; k < 4; ++k) s -= L[k][i] * x[k];
    x[i] = s * rd[i];
  }
  return true;
}

// Gaussian fit of one CCF held by the calling wave (y[t] = CCF point
// lane + 64 t); returns the result record and leaves the parameters in p and
// the last sums (gf_eval) in S.  Damped Newton / Levenberg-Marquardt as
// described at k_ccf_fit.
template <int NPT>
__device__ soap_rv fit_wave(const double (&y)[NPT], int n_v, double v0, double dv, double p[4],
                            double S[20]) {
  const int lane = threadIdx.x & 63;
  // start values: max, first argmin, half-depth width
  double ymax = -1e308, ymin = 1e308;
  int kmin = n_v;
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    const int i = lane + 64 * t;
    if (i < n_v) {
      ymax = fmax(ymax, y[t]);
      if (y[t] < ymin) {
        ymin = y[t];
        kmin = i;
      }
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
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    const int i = lane + 64 * t;
    if (i < n_v && y[t] <= half) {
      first = min(first, i);
      last = max(last, i);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    first = min(first, __shfl_xor(first, off, 64));
    last = max(last, __shfl_xor(last, off, 64));
  }
  // sample i of the CCF in every lane (i uniform, 0 <= i < n_v)
  auto at = [&](int i) {
    double v = y[0];
#pragma unroll
    for (int t = 1; t < NPT; ++t)
      if ((i >> 6) == t) v = y[t];
    return __shfl(v, i & 63, 64);
  };
  // half-depth crossings interpolated between samples, and the minimum's
  // position from the parabola through it and its neighbours
  double xl = first, xr = last;
  if (first > 0 && first < n_v) {
    const double ya = at(first - 1), yb = at(first);
    if (ya > yb) xl = (first - 1) + (ya - half) / (ya - yb);
  }
  if (last >= 0 && last + 1 < n_v) {
    const double ya = at(last), yb = at(last + 1);
    if (yb > ya) xr = last + (half - ya) / (yb - ya);
  }
  double kc = kmin;
  if (kmin > 0 && kmin + 1 < n_v) {
    const double ym = at(kmin - 1), y0 = at(kmin), yp = at(kmin + 1);
    const double den = ym - 2.0 * y0 + yp;
    if (den > 0.0) kc += fmin(fmax(0.5 * (ym - yp) / den, -0.5), 0.5);
  }
  const double width = (xr > xl) ? dv * (xr - xl) : dv;
  p[0] = c0;
  p[1] = a0;
  p[2] = v0 + dv * kc;
  p[3] = fmax(width, dv) / FWHM_PER_SIGMA;

  // every sample finite: max and min skip NaN, so test each one
  bool bad_sample = false;
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    const int i = lane + 64 * t;
    if (i < n_v && !isfinite(y[t])) bad_sample = true;
  }
  const bool any_bad = __ballot(bad_sample) != 0ull;

  soap_rv res;
  res.status = 0;
  if (any_bad || !(a0 > 1e-12 * fabs(c0)) || !isfinite(c0) || !isfinite(ymin)) {
    res.status = 2;
    res.iters = 0;
  } else {
    gf_eval(y, n_v, v0, dv, p, S);
    double lam = 1e-3;
    int it = 0, accepted = 0;
    res.status = 1;
    for (; it < 100; ++it) {
      double x[4];
      double Sn[20];
      bool ok = gf_solve(S, true, lam, x) || gf_solve(S, false, lam, x);
      bool tiny = false;
      if (ok) {
        const double sig = fabs(p[3]);
        tiny = fabs(x[0]) <= 1e-10 * fabs(p[0]) && fabs(x[1]) <= 1e-10 * fabs(p[1]) &&
               fabs(x[2]) <= 1e-10 * sig && fabs(x[3]) <= 1e-10 * sig;
        if (tiny) {
          // a step of rounding size: take it without another pass (chi2
          // stays that of the last evaluated point)
          for (int q = 0; q < 4; ++q) p[q] += x[q];
          res.status = 0;
          ++it;
          break;
        }
        double pn[4];
        for (int q = 0; q < 4; ++q) pn[q] = p[q] + x[q];
        gf_eval(y, n_v, v0, dv, pn, Sn);
        if (Sn[0] <= S[0]) {
          const double dchi = S[0] - Sn[0];
          for (int q = 0; q < 4; ++q) p[q] = pn[q];
          for (int q = 0; q < 20; ++q) S[q] = Sn[q];
          ++accepted;
          lam = (lam > 1e-9) ? lam * 0.1 : 0.0;
          const double sgn = fabs(p[3]);
          const bool floor_hit =
              dchi <= 1e-15 * S[0] && fabs(x[2]) <= 1e-9 * sgn && fabs(x[3]) <= 1e-9 * sgn;
          if (tiny || floor_hit) {
            res.status = 0;
            ++it;
            break;
          }
          continue;
        }
      }
      if (tiny) {  // a rounding-size step that does not lower chi^2
        res.status = 0;
        ++it;
        break;
      }
      lam = (lam > 0.0) ? lam * 10.0 : 1e-6;
      if (lam > 1e10) {
        // No damped step lowers chi^2.  That is the minimum at this
        // precision only when the point came from an accepted step and the
        // undamped Newton step there is of rounding size (at most 1e-7 of
        // each parameter's scale) or predicts a decrease of chi^2 / 2 below
        // 1e-12 of chi^2; otherwise (singular or non-finite sums, no step
        // ever accepted) the fit failed.
        bool conv = false;
        double xn[4];
        if (accepted > 0 && (gf_solve(S, true, 0.0, xn) || gf_solve(S, false, 0.0, xn))) {
          const double sg = fabs(p[3]);
          const bool small = fabs(xn[0]) <= 1e-7 * fabs(p[0]) && fabs(xn[1]) <= 1e-7 * fabs(p[1]) &&
                             fabs(xn[2]) <= 1e-7 * sg && fabs(xn[3]) <= 1e-7 * sg;
          const double dec = -0.5 * (S[1] * xn[0] + S[2] * xn[1] + S[3] * xn[2] + S[4] * xn[3]);
          conv = small || (isfinite(dec) && dec <= 1e-12 * S[0]);
        }
        res.status = conv ? 0 : 3;
        ++it;
        break;
      }
    }
    res.iters = it;
    res.chi2 = S[0];
  }
  res.rv_kms = p[2];
  res.sigma_kms = fabs(p[3]);
  res.fwhm_kms = FWHM_PER_SIGMA * fabs(p[3]);
  res.c0 = p[0];
  res.amp = p[1];
  if (res.status == 2) res.chi2 = 0.0;
  return res;
}

}  // namespace

// One block of four waves per spectrum.  The waves first add the line
// blocks' partial CCFs (wave w takes the line blocks lb = w mod 4, in
// order; the four partial sums are then added in wave order, so the result
// repeats bit for bit) and write the CCF.  With fit set, wave 0 then fits
// the Gaussian.
//
// Fit: damped Newton / Levenberg-Marquardt.  The step solves
// (H + lam diag(J^T J)) x = -J^T r with H the full Hessian of chi^2 / 2
// (J^T J plus the residual-weighted second derivatives; the CCF is not an
// exact Gaussian, so the residuals stay finite and Gauss-Newton alone
// converges only linearly) and falls back to H = J^T J where the full one
// is not positive definite.  A trial step is evaluated with all its sums,
// so an accepted step costs one pass over the CCF.  The fit has converged
// when a step moves every parameter by at most 1e-10 of its scale (sigma
// for the centre and width; at that size its chi^2 only reflects rounding,
// so it is taken without a pass), or when an accepted step no longer lowers
// chi^2 and moves the centre and width by at most 1e-9 sigma; a run of
// rejected steps that drives the damping past 1e10 means no downhill step
// exists at this precision, which is the minimum only when an earlier step
// was accepted and the undamped Newton step there is of rounding size
// (status 0); otherwise the fit failed (status 3).  A CCF with a non-finite
// sample or no depth is degenerate (status 2).
template <int NPT, typename PT>
__device__ __forceinline__ void fit_block(int n_lb, int64_t n_spec, int n_v, double v0, double dv,
                                          const PT* __restrict__ part, double* __restrict__ ccf, int fit,
                                          soap_rv* __restrict__ out, int64_t s) {
  __shared__ double s_sum[CCF_FIN_THREADS / 64][NPT * 64];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  constexpr int NW = CCF_FIN_THREADS / 64;
  constexpr int RB = (NPT <= 3 ? 16 : (NPT <= 6 ? 8 : 4)) / (sizeof(PT) == 8 ? 2 : 1);  // rows in flight per wave
  {
    double acc[NPT];
#pragma unroll
    for (int t = 0; t < NPT; ++t) acc[t] = 0.0;
    for (int lb0 = wave; lb0 < n_lb; lb0 += RB * NW) {
      double v[RB][NPT];
      // every load is unconditional (indices clamped into the rows) and the
      // out-of-range values are zeroed after it: loads under a branch would
      // each be waited for before the next one is issued
      PT raw[RB][NPT];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int lb = min(lb0 + u * NW, n_lb - 1);
        const PT* src = part + ((int64_t)lb * n_spec + s) * n_v;
#pragma unroll
        for (int t = 0; t < NPT; ++t) raw[u][t] = src[min(lane + 64 * t, n_v - 1)];
      }
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int lb = lb0 + u * NW;
#pragma unroll
        for (int t = 0; t < NPT; ++t) {
          const int i = lane + 64 * t;
          v[u][t] = (lb < n_lb && i < n_v) ? (double)raw[u][t] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < RB; ++u)
#pragma unroll
        for (int t = 0; t < NPT; ++t) acc[t] += v[u][t];
    }
#pragma unroll
    for (int t = 0; t < NPT; ++t) s_sum[wave][lane + 64 * t] = acc[t];
  }
  __syncthreads();
  if (wave != 0) return;
  double y[NPT];
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    const int i = lane + 64 * t;
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) a += s_sum[w][i];
    y[t] = a;
    if (i < n_v) ccf[s * n_v + i] = a;
  }
  if (!fit) return;
  double p[4], S[20];
  const soap_rv res = fit_wave(y, n_v, v0, dv, p, S);
  if (lane == 0) out[s] = res;
}

template <int NPT, typename PT>
__global__ void __launch_bounds__(CCF_FIN_THREADS) k_ccf_fit(int n_lb, int64_t n_spec, int n_v, double v0,
                                                             double dv, const PT* __restrict__ part,
                                                             double* __restrict__ ccf, int fit,
                                                             soap_rv* __restrict__ out) {
  fit_block<NPT, PT>(n_lb, n_spec, n_v, v0, dv, part, ccf, fit, out, blockIdx.x);
}

// One wave per spectrum: the same sums in the same order as fit_block's
// four waves (row lb goes to accumulator lb mod 4, rows ascending; the four
// accumulators are then added in order), so the CCF and the fit repeat
// fit_block's bit for bit; with every wave of a block fitting, four times as
// many fits are in flight.
template <int NPT, typename PT>
__device__ __forceinline__ void fit_one_wave(int n_lb, int64_t n_spec, int n_v, double v0, double dv,
                                             const PT* __restrict__ part, double* __restrict__ ccf, int fit,
                                             soap_rv* __restrict__ out, int64_t s) {
  const int lane = threadIdx.x & 63;
  constexpr int NW = CCF_FIN_THREADS / 64;  // fit_block's interleave of line blocks
  constexpr int RB = 2 * NW;                // rows in flight, a multiple of NW
  double acc[NW][NPT];
#pragma unroll
  for (int w = 0; w < NW; ++w)
#pragma unroll
    for (int t = 0; t < NPT; ++t) acc[w][t] = 0.0;
  for (int lb0 = 0; lb0 < n_lb; lb0 += RB) {
    // unconditional loads (indices clamped), out-of-range values zeroed after
    PT raw[RB][NPT];
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int lb = min(lb0 + u, n_lb - 1);
      const PT* src = part + ((int64_t)lb * n_spec + s) * n_v;
#pragma unroll
      for (int t = 0; t < NPT; ++t) raw[u][t] = src[min(lane + 64 * t, n_v - 1)];
    }
#pragma unroll
    for (int u = 0; u < RB; ++u)
#pragma unroll
      for (int t = 0; t < NPT; ++t) {
        const int i = lane + 64 * t;
        acc[u % NW][t] += (lb0 + u < n_lb && i < n_v) ? (double)raw[u][t] : 0.0;
      }
  }
  double y[NPT];
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    const int i = lane + 64 * t;
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) a += acc[w][t];
    y[t] = a;
    if (i < n_v) ccf[s * n_v + i] = a;
  }
  if (!fit) return;
  double p[4], S[20];
  const soap_rv res = fit_wave(y, n_v, v0, dv, p, S);
  if (lane == 0) out[s] = res;
}

// One wave per spectrum over one spectra set (calls with many spectra).
template <int NPT, typename PT>
__global__ void __launch_bounds__(CCF_FIN_THREADS) k_ccf_fit_waves(int n_lb, int64_t n_spec, int n_v, double v0,
                                                                   double dv, const PT* __restrict__ part,
                                                                   double* __restrict__ ccf, int fit,
                                                                   soap_rv* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * (CCF_FIN_THREADS / 64) + (threadIdx.x >> 6);
  if (s >= n_spec) return;  // whole waves
  fit_one_wave<NPT, PT>(n_lb, n_spec, n_v, v0, dv, part, ccf, fit, out, s);
}

// Work-list form, one wave per entry: blk[b] = (set, spectrum).
template <int NPT, typename PT>
__global__ void __launch_bounds__(CCF_FIN_THREADS) k_ccf_fit_batch(const CcfBatchSet* __restrict__ sets,
                                                                   const int2* __restrict__ blk, int n_blk, int n_v,
                                                                   double v0, double dv) {
  const int b = blockIdx.x * (CCF_FIN_THREADS / 64) + (threadIdx.x >> 6);
  if (b >= n_blk) return;  // whole waves
  const int2 t = blk[b];
  const CcfBatchSet c = sets[t.x];
  fit_one_wave<NPT, PT>(c.nlb, c.n_spec, n_v, v0, dv, static_cast<const PT*>(c.part), c.ccf, c.rv ? 1 : 0, c.rv,
                        t.y);
}

template <typename T, int A, int NPX, int STG>
static void launch_ccf_a(const CcfPlan& q, hipStream_t st, dim3 grid, const void* d_flux, int64_t n_spec,
                         void* d_part) {
  const unsigned char* base = q.tables;
  hipLaunchKernelGGL((k_ccf<T, A, NPX, STG>), grid, dim3(CCF_THREADS), 0, st, (int)q.P, n_spec,
                     static_cast<const T*>(d_flux), reinterpret_cast<const double2*>(base),
                     reinterpret_cast<const double2*>(base + q.off_edges),
                     reinterpret_cast<const int4*>(base + q.off_batch),
                     reinterpret_cast<const int*>(base + q.off_bfirst), q.nv, static_cast<T*>(d_part));
}

template <typename T, int NPX, int STG>
static void launch_ccf_n(const CcfPlan& q, hipStream_t st, dim3 grid, const void* d_flux, int64_t n_spec,
                         void* d_part) {
  if (q.nv <= CCF_THREADS) launch_ccf_a<T, 1, NPX, STG>(q, st, grid, d_flux, n_spec, d_part);
  else if (q.nv <= 2 * CCF_THREADS) launch_ccf_a<T, 2, NPX, STG>(q, st, grid, d_flux, n_spec, d_part);
  else launch_ccf_a<T, 4, NPX, STG>(q, st, grid, d_flux, n_spec, d_part);
}

template <typename T, int STG>
static void launch_ccf_s(const CcfPlan& q, hipStream_t st, dim3 grid, const void* d_flux, int64_t n_spec,
                         void* d_part) {
  switch (q.npx) {
    case 2: launch_ccf_n<T, 2, STG>(q, st, grid, d_flux, n_spec, d_part); break;
    case 3: launch_ccf_n<T, 3, STG>(q, st, grid, d_flux, n_spec, d_part); break;
    case 5: launch_ccf_n<T, 5, STG>(q, st, grid, d_flux, n_spec, d_part); break;
    default: launch_ccf_n<T, 10, STG>(q, st, grid, d_flux, n_spec, d_part); break;
  }
}

template <typename T>
static void launch_ccf_t(const CcfPlan& q, hipStream_t st, dim3 grid, const void* d_flux, int64_t n_spec,
                         void* d_part) {
  if (q.stg <= 256) launch_ccf_s<T, 256>(q, st, grid, d_flux, n_spec, d_part);
  else launch_ccf_s<T, CCF_STG_MAX>(q, st, grid, d_flux, n_spec, d_part);
}

CcfPlan ccf_plan(const soap_ctx* c, int n_lines, const void* tables) {
  CcfPlan q;
  q.tables = static_cast<const unsigned char*>(tables);
  q.off_edges = c->ccf_off_edges;
  q.off_batch = c->ccf_off_batch;
  q.off_bfirst = c->ccf_off_bfirst;
  q.npx = c->ccf_npx;
  q.stg = c->ccf_stg;
  q.nv = c->mask_nv;
  q.n_lines = n_lines;
  q.v0 = c->mask_v0;
  q.dv = c->mask_dv;
  q.fp32 = c->prec == SOAP_PREC_FP32;
  q.P = c->P;
  return q;
}

hipError_t launch_ccf_p(const CcfPlan& q, hipStream_t st, const void* d_flux, int64_t n_spec, void* d_part) {
  const int nlb = ccf_line_blocks(q.n_lines);
  dim3 grid(nlb, (unsigned)((n_spec + CCF_SB - 1) / CCF_SB));
  if (q.fp32) launch_ccf_t<float>(q, st, grid, d_flux, n_spec, d_part);
  else launch_ccf_t<double>(q, st, grid, d_flux, n_spec, d_part);
  return hipGetLastError();
}

hipError_t launch_ccf(soap_ctx* c, const void* d_flux, int64_t n_spec, int n_lines, void* d_part) {
  return launch_ccf_p(ccf_plan(c, n_lines, c->ws_mask.ptr), c->stream, d_flux, n_spec, d_part);
}

// the fit kernel for the mask's points per lane
template <typename PT>
static hipError_t launch_fit_npt(const CcfPlan& q, hipStream_t st, int nlb, int64_t n_spec, const PT* d_part,
                                 double* d_ccf, soap_rv* d_rv) {
  const int npt = (q.nv + 63) / 64;
  // up to CCF_FIT_WAVES_FROM spectra a block of four waves per spectrum
  // (partial sums spread over the block, every fit in flight at once);
  // beyond, a wave per spectrum (four fits in flight per block); both give
  // the same records bit for bit
  constexpr int kWaves = CCF_FIN_THREADS / 64;
  const bool waves = n_spec > CCF_FIT_WAVES_FROM;
  const unsigned grid = waves ? (unsigned)((n_spec + kWaves - 1) / kWaves) : (unsigned)n_spec;
#define FIT_CASE(N)                                                                                          \
  case N:                                                                                                    \
    if (waves)                                                                                               \
      hipLaunchKernelGGL((k_ccf_fit_waves<N, PT>), dim3(grid), dim3(CCF_FIN_THREADS), 0, st, nlb, n_spec, q.nv, \
                         q.v0, q.dv, d_part, d_ccf, d_rv ? 1 : 0, d_rv);                                     \
    else                                                                                                     \
      hipLaunchKernelGGL((k_ccf_fit<N, PT>), dim3(grid), dim3(CCF_FIN_THREADS), 0, st, nlb, n_spec, q.nv, q.v0, \
                         q.dv, d_part, d_ccf, d_rv ? 1 : 0, d_rv);                                           \
    break;
  switch (npt) {
    FIT_CASE(1) FIT_CASE(2) FIT_CASE(3) FIT_CASE(4) FIT_CASE(5) FIT_CASE(6)
    FIT_CASE(7) FIT_CASE(8) FIT_CASE(9) FIT_CASE(10) FIT_CASE(11) FIT_CASE(12)
    default: return hipErrorInvalidValue;
  }
#undef FIT_CASE
  return hipGetLastError();
}

hipError_t launch_ccf_fit_p(const CcfPlan& q, hipStream_t st, const void* d_part, int64_t n_spec, double* d_ccf,
                            soap_rv* d_rv) {
  const int nlb = ccf_line_blocks(q.n_lines);
  if (q.fp32) return launch_fit_npt(q, st, nlb, n_spec, static_cast<const float*>(d_part), d_ccf, d_rv);
  return launch_fit_npt(q, st, nlb, n_spec, static_cast<const double*>(d_part), d_ccf, d_rv);
}

hipError_t launch_ccf_fit(soap_ctx* c, int n_lines, const void* d_part, int64_t n_spec, double* d_ccf,
                          soap_rv* d_rv) {
  return launch_ccf_fit_p(ccf_plan(c, n_lines, c->ws_mask.ptr), c->stream, d_part, n_spec, d_ccf, d_rv);
}

// ---- work-list CCF + fit over many spectra sets ------------------------------

bool ccf_same_layout(const CcfPlan& a, const CcfPlan& b) {
  return a.fp32 == b.fp32 && a.npx == b.npx && (a.stg <= 256) == (b.stg <= 256) && a.nv == b.nv && a.v0 == b.v0 &&
         a.dv == b.dv;
}

namespace {

size_t al256c(size_t b) { return 256 * ((b + 255) / 256); }

template <typename T, int A, int NPX, int STG>
void launch_ccf_batch_a(const CcfBatch& cb, hipStream_t st) {
  hipLaunchKernelGGL((k_ccf_batch<T, A, NPX, STG>), dim3((unsigned)cb.n_ccf_blocks), dim3(CCF_THREADS), 0, st,
                     cb.sets, cb.ccf_blk, cb.shape.nv);
}

template <typename T, int NPX, int STG>
void launch_ccf_batch_n(const CcfBatch& cb, hipStream_t st) {
  if (cb.shape.nv <= CCF_THREADS) launch_ccf_batch_a<T, 1, NPX, STG>(cb, st);
  else if (cb.shape.nv <= 2 * CCF_THREADS) launch_ccf_batch_a<T, 2, NPX, STG>(cb, st);
  else launch_ccf_batch_a<T, 4, NPX, STG>(cb, st);
}

template <typename T, int STG>
void launch_ccf_batch_s(const CcfBatch& cb, hipStream_t st) {
  switch (cb.shape.npx) {
    case 2: launch_ccf_batch_n<T, 2, STG>(cb, st); break;
    case 3: launch_ccf_batch_n<T, 3, STG>(cb, st); break;
    case 5: launch_ccf_batch_n<T, 5, STG>(cb, st); break;
    default: launch_ccf_batch_n<T, 10, STG>(cb, st); break;
  }
}

template <typename T>
void launch_ccf_batch_t(const CcfBatch& cb, hipStream_t st) {
  if (cb.shape.stg <= 256) launch_ccf_batch_s<T, 256>(cb, st);
  else launch_ccf_batch_s<T, CCF_STG_MAX>(cb, st);
}

template <typename PT>
hipError_t launch_fit_batch_pt(const CcfBatch& cb, hipStream_t st) {
  const int npt = (cb.shape.nv + 63) / 64;
  constexpr int kWaves = CCF_FIN_THREADS / 64;  // one spectrum per wave
  const unsigned grid = (unsigned)((cb.n_fit_blocks + kWaves - 1) / kWaves);
#define FITB_CASE(N)                                                                                           \
  case N:                                                                                                      \
    hipLaunchKernelGGL((k_ccf_fit_batch<N, PT>), dim3(grid), dim3(CCF_FIN_THREADS), 0, st, cb.sets, cb.fit_blk, \
                       cb.n_fit_blocks, cb.shape.nv, cb.shape.v0, cb.shape.dv);                                 \
    break;
  switch (npt) {
    FITB_CASE(1) FITB_CASE(2) FITB_CASE(3) FITB_CASE(4) FITB_CASE(5) FITB_CASE(6)
    FITB_CASE(7) FITB_CASE(8) FITB_CASE(9) FITB_CASE(10) FITB_CASE(11) FITB_CASE(12)
    default: return hipErrorInvalidValue;
  }
#undef FITB_CASE
  return hipGetLastError();
}

}  // namespace

size_t ccf_batch_bytes(const CcfPlan* plans, const int64_t* n_spec, int n) {
  size_t ccf_blocks = 0, fit_blocks = 0;
  for (int i = 0; i < n; ++i) {
    ccf_blocks += (size_t)ccf_line_blocks(plans[i].n_lines) * (size_t)((n_spec[i] + CCF_SB - 1) / CCF_SB);
    fit_blocks += (size_t)n_spec[i];
  }
  return al256c(sizeof(CcfBatchSet) * n) + al256c(sizeof(int4) * ccf_blocks) + al256c(sizeof(int2) * fit_blocks);
}

hipError_t ccf_batch_upload(const CcfPlan* plans, const CcfBatchSet* sets, int n, void* d_buf, CcfBatch* cb) {
  if (n < 1) return hipErrorInvalidValue;
  std::vector<CcfBatchSet> hs(sets, sets + n);
  std::vector<int4> cblk;
  std::vector<int2> fblk;
  for (int i = 0; i < n; ++i) {
    if (!ccf_same_layout(plans[i], plans[0]) || sets[i].n_spec < 1 || sets[i].n_spec > (int64_t(1) << 24))
      return hipErrorInvalidValue;
    const CcfPlan& q = plans[i];
    CcfBatchSet& h = hs[i];
    h.P = (int)q.P;
    h.nlb = ccf_line_blocks(q.n_lines);
    h.tables = q.tables;
    h.off_edges = q.off_edges;
    h.off_batch = q.off_batch;
    h.off_bfirst = q.off_bfirst;
    const int nsb = (int)((h.n_spec + CCF_SB - 1) / CCF_SB);
    for (int lb = 0; lb < h.nlb; ++lb)
      for (int sb = 0; sb < nsb; ++sb) cblk.push_back(make_int4(i, lb, sb, 0));
    for (int64_t sp = 0; sp < h.n_spec; ++sp) fblk.push_back(make_int2(i, (int)sp));
  }
  unsigned char* base = static_cast<unsigned char*>(d_buf);
  cb->shape = plans[0];
  cb->n_sets = n;
  cb->n_ccf_blocks = (int)cblk.size();
  cb->n_fit_blocks = (int)fblk.size();
  cb->sets = reinterpret_cast<CcfBatchSet*>(base);
  size_t used = al256c(sizeof(CcfBatchSet) * n);
  cb->ccf_blk = reinterpret_cast<int4*>(base + used);
  used += al256c(sizeof(int4) * cblk.size());
  cb->fit_blk = reinterpret_cast<int2*>(base + used);
  hipError_t e = hipMemcpy(cb->sets, hs.data(), sizeof(CcfBatchSet) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(cb->ccf_blk, cblk.data(), sizeof(int4) * cblk.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(cb->fit_blk, fblk.data(), sizeof(int2) * fblk.size(), hipMemcpyHostToDevice);
  return e;
}

hipError_t ccf_batch_launch(const CcfBatch& cb, hipStream_t st) {
  if (cb.n_ccf_blocks <= 0) return hipSuccess;
  if (cb.shape.fp32) launch_ccf_batch_t<float>(cb, st);
  else launch_ccf_batch_t<double>(cb, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return cb.shape.fp32 ? launch_fit_batch_pt<float>(cb, st) : launch_fit_batch_pt<double>(cb, st);
}

// ccf[i][v] = base[v] + sum_k coef[i][k] basis[k][v] (double, increasing k):
// the CCF of a spectrum written in a basis, by linearity.  One block per row.
__global__ void __launch_bounds__(256) k_ccf_linear(int64_t n, int k, int n_v, const float* __restrict__ coef,
                                                    const double* __restrict__ base,
                                                    const double* __restrict__ basis, double* __restrict__ ccf) {
  __shared__ double s_c[256];
  const int64_t i = blockIdx.x;
  for (int v0 = 0; v0 < n_v; v0 += 256) {
    const int v = v0 + threadIdx.x;
    double a = v < n_v ? base[v] : 0.0;
    for (int k0 = 0; k0 < k; k0 += 256) {
      __syncthreads();
      if (k0 + (int)threadIdx.x < k) s_c[threadIdx.x] = (double)coef[i * k + k0 + threadIdx.x];
      __syncthreads();
      const int kn = min(256, k - k0);
      if (v < n_v)
        for (int j = 0; j < kn; ++j) a = fma(s_c[j], basis[(int64_t)(k0 + j) * n_v + v], a);
    }
    if (v < n_v) ccf[i * n_v + v] = a;
  }
}

constexpr int SG_MAX_ENS = 16;

// samples per wave of k_sg_lin and k_sg_spread (they share every basis row
// loaded) and basis rows in flight, by CCF points per lane
template <int NPT>
constexpr int sg_samples() {
  return NPT <= 3 ? 4 : (NPT <= 6 ? 2 : 1);
}
template <int NPT>
constexpr int sg_rows_in_flight() {
  return NPT <= 3 ? 8 : (NPT <= 6 ? 4 : 2);
}

// Surrogate RVs and their gate in three launches (so that each keeps few
// registers and many waves in flight):
//   k_sg_lin: CCF of the ensemble-mean prediction by linearity, base (the
//     sample's row base[base_idx[i]] when base_idx is given) + sum_k
//     coef[i][k] basis[k] (double, increasing k: the same sums as
//     k_ccf_linear), SS = sg_samples samples per wave sharing every basis
//     row loaded;
//   k_sg_fit: its Gaussian fit (fit_wave), one wave per sample, and the RV
//     sensitivity g = J H^-1 e_mu at the fit: the fitted parameters move by
//     dp = H^-1 J^T dy for a CCF change dy (H the Hessian of chi^2 / 2 at the
//     fit, J the model Jacobian), so dRV = g . dy;
//   k_sg_spread: each member's RV change dRV_e = sum_k h_k (y_e,k - coef_k)
//     with h = basis g (dy_e = sum_k (y_e,k - coef_k) basis[k]), SS samples
//     per wave; err = calib x the sample standard deviation of the dRV_e;
//     fallback when err is not below thr or the fit did not converge.
// Every sum of a sample keeps one fixed order.
template <int NPT>
__global__ void __launch_bounds__(64) k_sg_lin(int64_t n, int k, int n_v, const float* __restrict__ coef,
                                               const double* __restrict__ base, const int* __restrict__ base_idx,
                                               int n_base, const double* __restrict__ basis,
                                               double* __restrict__ Y, int* __restrict__ flag) {
  constexpr int SS = sg_samples<NPT>();
  constexpr int JU = sg_rows_in_flight<NPT>();
  __shared__ double s_c[SS][64];
  const int lane = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * SS;
  // Loads are unconditional, with indices clamped into the rows (lanes past
  // the grid and samples past n compute values that are never stored): a
  // load under a branch is waited for before the next one is issued.  A
  // sample whose star row does not exist reads row 0 and is flagged.
  int64_t ii[SS];
  bool row_ok[SS];
  const double* bs[SS];
#pragma unroll
  for (int s = 0; s < SS; ++s) {
    ii[s] = min(i0 + s, n - 1);
    const int brow = base_idx ? base_idx[ii[s]] : 0;
    row_ok[s] = brow >= 0 && brow < n_base;
    bs[s] = base + (int64_t)(row_ok[s] ? brow : 0) * n_v;
  }
  int vc[NPT];
#pragma unroll
  for (int t = 0; t < NPT; ++t) vc[t] = min(lane + 64 * t, n_v - 1);
  double y[SS][NPT];
#pragma unroll
  for (int s = 0; s < SS; ++s)
#pragma unroll
    for (int t = 0; t < NPT; ++t) y[s][t] = bs[s][vc[t]];
  for (int k0 = 0; k0 < k; k0 += 64) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < SS; ++s) s_c[s][lane] = k0 + lane < k ? (double)coef[ii[s] * k + min(k0 + lane, k - 1)] : 0.0;
    __syncthreads();
    const int kn = min(64, k - k0);
    for (int j0 = 0; j0 < kn; j0 += JU) {
      double b[JU][NPT];
#pragma unroll
      for (int u = 0; u < JU; ++u) {
        const double* bj = basis + (int64_t)(k0 + min(j0 + u, kn - 1)) * n_v;
#pragma unroll
        for (int t = 0; t < NPT; ++t) b[u][t] = bj[vc[t]];
      }
#pragma unroll
      for (int u = 0; u < JU; ++u)
#pragma unroll
        for (int s = 0; s < SS; ++s) {
          const double cj = j0 + u < kn ? s_c[s][j0 + u] : 0.0;  // rows past kn add zero
#pragma unroll
          for (int t = 0; t < NPT; ++t) y[s][t] = fma(cj, b[u][t], y[s][t]);
        }
    }
  }
#pragma unroll
  for (int s = 0; s < SS; ++s) {
    if (i0 + s >= n) break;
#pragma unroll
    for (int t = 0; t < NPT; ++t) {
      const int v = lane + 64 * t;
      if (v < n_v) Y[(i0 + s) * n_v + v] = y[s][t];
    }
    if (lane == 0) flag[i0 + s] = row_ok[s] ? 0 : 1;
  }
}

// flag[i] on entry: 1 when the sample has no star row; on exit: 1 when it
// has no surrogate RV (no row, or the fit or its sensitivity failed).
template <int NPT>
__global__ void __launch_bounds__(64) k_sg_fit(int64_t n, int n_v, double v0, double dv,
                                               const double* __restrict__ Y, int* __restrict__ flag,
                                               soap_rv* __restrict__ out, double* __restrict__ rv_kms,
                                               double* __restrict__ G) {
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  const bool row_ok = flag[i] == 0;
  double y[NPT];
#pragma unroll
  for (int t = 0; t < NPT; ++t) y[t] = Y[i * n_v + min(lane + 64 * t, n_v - 1)];
  double p[4], S[20];
  soap_rv res = fit_wave(y, n_v, v0, dv, p, S);
  bool bad = res.status != 0 || !row_ok;
  double z[4] = {0.0, 0.0, 0.0, 0.0};
  if (!bad) {
    // z = H^-1 e_mu (full Hessian; J^T J where that is not positive definite)
    double Sz[20];
#pragma unroll
    for (int q = 0; q < 20; ++q) Sz[q] = S[q];
    Sz[1] = 0.0;
    Sz[2] = 0.0;
    Sz[3] = -1.0;  // gf_solve solves A x = -S[1..4]
    Sz[4] = 0.0;
    if (!(gf_solve(Sz, true, 0.0, z) || gf_solve(Sz, false, 0.0, z))) bad = true;
  }
  const double is = 1.0 / p[3];
  const double is2 = is * is;
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    const int v = lane + 64 * t;
    if (v < n_v) {
      const double d = v0 + dv * v - p[2];
      const double zz = d * d * is2;
      const double e = exp(-0.5 * zz);
      const double ae = p[1] * e;
      G[i * n_v + v] = bad ? 0.0 : z[0] - e * z[1] - ae * d * is2 * z[2] - ae * zz * is * z[3];
    }
  }
  if (lane == 0) {
    if (!row_ok) {
      res = soap_rv{};
      res.status = 2;
    }
    if (out) out[i] = res;
    rv_kms[i] = row_ok ? res.rv_kms : 0.0;
    flag[i] = bad ? 1 : 0;
  }
}

template <int NPT, int EB>
__global__ void __launch_bounds__(64) k_sg_spread(int64_t n, int k, int E, int n_v, const float* __restrict__ coef,
                                                  const float* __restrict__ members,
                                                  const double* __restrict__ basis, const double* __restrict__ G,
                                                  const int* __restrict__ flag, double calib, double thr,
                                                  double* __restrict__ err_kms, int* __restrict__ fallback) {
  constexpr int SS = sg_samples<NPT>();
  __shared__ double s_g[SS][NPT * 64];
  const int lane = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * SS;
  int64_t ii[SS];
  bool bad[SS];
#pragma unroll
  for (int s = 0; s < SS; ++s) {
    ii[s] = min(i0 + s, n - 1);
    bad[s] = flag[ii[s]] != 0;
#pragma unroll
    for (int t = 0; t < NPT; ++t) {
      const int v = lane + 64 * t;
      if (v < n_v) s_g[s][v] = G[ii[s] * n_v + v];
    }
  }
  __syncthreads();
  // h_k = sum_v basis[k][v] g_v, then dRV_e = sum_k h_k (y_e,k - coef_k)
  double dr[SS][EB];
#pragma unroll
  for (int s = 0; s < SS; ++s)
#pragma unroll
    for (int e = 0; e < EB; ++e) dr[s][e] = 0.0;
  for (int k0 = 0; k0 < k; k0 += 64) {
    const int kk = k0 + lane;
    const int kc = min(kk, k - 1);
    const double* bk = basis + (int64_t)kc * n_v;
    // four partial sums over v per sample (16 samples of the row in flight),
    // added in a fixed order
    double h4[SS][4];
#pragma unroll
    for (int s = 0; s < SS; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q) h4[s][q] = 0.0;
    int v = 0;
    for (; v + 16 <= n_v; v += 16) {
      double bv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) bv[u] = bk[v + u];
#pragma unroll
      for (int s = 0; s < SS; ++s)
#pragma unroll
        for (int u = 0; u < 16; ++u) h4[s][u & 3] = fma(bv[u], s_g[s][v + u], h4[s][u & 3]);
    }
    for (; v < n_v; ++v) {
      const double bvv = bk[v];
#pragma unroll
      for (int s = 0; s < SS; ++s) h4[s][0] = fma(bvv, s_g[s][v], h4[s][0]);
    }
#pragma unroll
    for (int s = 0; s < SS; ++s) {
      const double h = kk < k ? (h4[s][0] + h4[s][1]) + (h4[s][2] + h4[s][3]) : 0.0;
      const double cm = (double)coef[ii[s] * k + kc];
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        if (e < E) {
          const double ye = (double)members[((int64_t)e * n + ii[s]) * k + kc];
          dr[s][e] += h * (ye - cm);
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < SS; ++s) {
    double err = 0.0;
    if (!bad[s]) {
      double m = 0.0;
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        if (e < E) {  // uniform
          dr[s][e] = wave_sum_f64(dr[s][e]);
          m += dr[s][e];
        }
      }
      m /= (double)E;
      double var = 0.0;
#pragma unroll
      for (int e = 0; e < EB; ++e)
        if (e < E) var += (dr[s][e] - m) * (dr[s][e] - m);
      err = calib * sqrt(var / (double)(E - 1));
    }
    if (lane == 0 && i0 + s < n) {
      if (err_kms) err_kms[i0 + s] = bad[s] ? INFINITY : err;
      fallback[i0 + s] = (bad[s] || !(err < thr)) ? 1 : 0;
    }
  }
}

namespace {

template <int NPT>
void launch_sg_rv_n(soap_ctx* c, const float* d_coef, const float* d_members, int64_t n, int E, int k,
                    const double* d_base, const int* d_base_idx, int n_base, const double* d_basis, double calib,
                    double thr, soap_rv* d_rv, double* d_rv_kms, double* d_err, int* d_fallback, double* Y,
                    double* G, int* flag) {
  const dim3 grid_s((unsigned)((n + sg_samples<NPT>() - 1) / sg_samples<NPT>())), block(64);
  const int nb = d_base_idx ? n_base : 1;
  hipLaunchKernelGGL((k_sg_lin<NPT>), grid_s, block, 0, c->stream, n, k, c->mask_nv, d_coef, d_base, d_base_idx, nb,
                     d_basis, Y, flag);
  hipLaunchKernelGGL((k_sg_fit<NPT>), dim3((unsigned)n), block, 0, c->stream, n, c->mask_nv, c->mask_v0,
                     c->mask_dv, Y, flag, d_rv, d_rv_kms, G);
  if (E <= 4)
    hipLaunchKernelGGL((k_sg_spread<NPT, 4>), grid_s, block, 0, c->stream, n, k, E, c->mask_nv, d_coef, d_members,
                       d_basis, G, flag, calib, thr, d_err, d_fallback);
  else if (E <= 8)
    hipLaunchKernelGGL((k_sg_spread<NPT, 8>), grid_s, block, 0, c->stream, n, k, E, c->mask_nv, d_coef, d_members,
                       d_basis, G, flag, calib, thr, d_err, d_fallback);
  else
    hipLaunchKernelGGL((k_sg_spread<NPT, SG_MAX_ENS>), grid_s, block, 0, c->stream, n, k, E, c->mask_nv, d_coef,
                       d_members, d_basis, G, flag, calib, thr, d_err, d_fallback);
}

}  // namespace

hipError_t launch_sg_rv(soap_ctx* c, const float* d_coef, const float* d_members, int64_t n, int E, int k,
                        const double* d_base, const int* d_base_idx, int n_base, const double* d_basis,
                        double calib, double thr, soap_rv* d_rv, double* d_rv_kms, double* d_err,
                        int* d_fallback, void* d_work) {
  if (E < 2 || E > SG_MAX_ENS) return hipErrorInvalidValue;
  const int npt = (c->mask_nv + 63) / 64;
  double* Y = static_cast<double*>(d_work);
  double* G = Y + (size_t)n * c->mask_nv;
  int* flag = reinterpret_cast<int*>(G + (size_t)n * c->mask_nv);
#define SG_CASE(N)                                                                                              \
  case N:                                                                                                       \
    launch_sg_rv_n<N>(c, d_coef, d_members, n, E, k, d_base, d_base_idx, n_base, d_basis, calib, thr, d_rv,     \
                      d_rv_kms, d_err, d_fallback, Y, G, flag);                                                 \
    break;
  switch (npt) {
    SG_CASE(1) SG_CASE(2) SG_CASE(3) SG_CASE(4) SG_CASE(5) SG_CASE(6)
    SG_CASE(7) SG_CASE(8) SG_CASE(9) SG_CASE(10) SG_CASE(11) SG_CASE(12)
    default: return hipErrorInvalidValue;
  }
#undef SG_CASE
  return hipGetLastError();
}

size_t sg_rv_work_bytes(const soap_ctx* c, int64_t n) {
  return sizeof(double) * 2 * (size_t)n * c->mask_nv + sizeof(int) * (size_t)n;
}

hipError_t launch_ccf_linear_fit(soap_ctx* c, const float* d_coef, int64_t n, int k, const double* d_base,
                                 const double* d_basis, double* d_lin, double* d_ccf, soap_rv* d_rv) {
  hipLaunchKernelGGL(k_ccf_linear, dim3((unsigned)n), dim3(256), 0, c->stream, n, k, c->mask_nv, d_coef, d_base,
                     d_basis, d_lin);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the rows are complete CCFs: one "block of lines" for the fit kernel
  return launch_fit_npt(ccf_plan(c, 1, c->ws_mask.ptr), c->stream, 1, n, d_lin, d_ccf, d_rv);
}



}  // namespace soap
