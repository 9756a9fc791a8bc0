// Per-phase active-region weights (section 3.3, Algorithm 5).
//
// k_weights: one block per (phase, slab of SLAB_COLS disk columns), flattened
//   1. rotates every region centre to the phase (longitude + 360 deg * phase,
//      axis tilted by the inclination) and bounds the visible caps;
//   2. one wave64 per column, one lane per cell: a cell belongs to a region
//      when the angle between its surface point and the region centre is at
//      most asin(radius); the InfoMap owner is the last listed region that
//      covers it;
//   3. per column, the weights A I(mu) of the active cells are summed per
//      (type, mu bin): each lane sums its own cells (FP32 + Kahan in the
//      FP32 mode, FP64 otherwise) and adds each sum to a per-wave LDS table
//      as an exact 64-bit fixed-point integer;
//   4. each column sum is collapsed onto the two integer offsets of the
//      column's shift (1 - w at j = c, w at j = c - 1: Eq. 11).
// Tables: paired mode (every active weight equals its removal weight:
// chromatic contrast, the convective effect, or unit scalar contrasts) keeps
// one table row per active (type, bin), g = (type - 1) * B + bin, and the
// quiet removal is implied by the apply kernel.  Split mode (scalar
// contrasts other than one) keeps g = type * B + bin with type 0 the removal
// (-A I) and the active rows scaled by the region contrast.
//
// Column contributions go straight to per-phase tap tables in 64-bit fixed
// point (exact integer atomics, so the totals repeat bit for bit whatever
// the order).  k_finish, one block per chunk of phases, converts the tables
// to double (clearing them for the next call), records per (phase, group)
// the bitmask of non-zero offsets, and turns the chunk into window records
// of APPLY_JW offsets with dense taps and per-offset masks of the pairs of
// phases that have a tap.
// Every sum has a fixed order, so results repeat bit for bit.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "soap_internal.hpp"
#include "wave.hpp"

namespace soap {

namespace {


constexpr int MAXC = 4;   // cells per lane per row pass (256 rows)

// taps are accumulated as 64-bit fixed point in units of 2^-59 (|tap| < 16):
// integer addition is exact, so the totals do not depend on the order in
// which columns arrive
__device__ __forceinline__ unsigned long long to_fx(double x) {
  return (unsigned long long)__double2ll_rn(x * FX_ONE);
}

}  // namespace

// Window records of one chunk of PC phases (one block): windows of APPLY_JW
// offsets with their dense [offset][phase] taps and per-offset masks of the
// pairs of phases that have a tap.  Kc: the chunk's taps [np][G][J],
// maskc: its offset masks [np][G] (LDS or global).  sm: LDS of at least
// (4 G + vg_cap + 2) ints + G 64-bit words.
template <typename T>
__device__ void compact_chunk(int chunk, int n_ph, int PC, int G, int J, int jmin, int B, int paired,
                              const double* Kc, const unsigned long long* maskc, unsigned char* __restrict__ wins,
                              int* __restrict__ nvg, int vg_cap, int* sm) {
  int* s_cnt = sm;           // [G] windows per group
  int* s_base = sm + G;      // [G] first window index
  int* s_lo = sm + 2 * G;    // [G] first non-zero offset of the union
  int* s_nv = sm + 3 * G;    // [1]
  unsigned int* s_gm = reinterpret_cast<unsigned int*>(sm + 4 * G);  // [vg_cap] group masks
  unsigned long long* s_union = reinterpret_cast<unsigned long long*>(sm + 4 * G + vg_cap + (vg_cap & 1));  // [G]
  const int p0 = chunk * PC;
  const int np = min(PC, n_ph - p0);
  const int NP = PC / 2;  // mask bits per offset: pairs of phases
  const int GJ = G * J;
  const int nwin = (J + APPLY_JW - 1) / APPLY_JW;
  const int wb = win_bytes(PC, (int)sizeof(T));  // record bytes
  unsigned char* wrec = wins + (int64_t)chunk * vg_cap * wb;

  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    unsigned long long u = 0;
#pragma unroll
    for (int p = 0; p < PC_MAX; ++p)
      if (p < np) u |= maskc[p * G + g];
    int cnt = 0, lo = 0;
    if (u) {
      lo = __builtin_ctzll(u);
      for (int a = lo; a < J; a += APPLY_JW)
        if ((u >> a) & ((1ull << APPLY_JW) - 1)) ++cnt;
    }
    s_cnt[g] = cnt;
    s_lo[g] = lo;
    s_union[g] = u;
  }
  for (int v = threadIdx.x; v < vg_cap; v += blockDim.x) s_gm[v] = 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int g = 0; g < G; ++g) {
      s_base[g] = acc;
      acc += s_cnt[g];
    }
    nvg[chunk] = acc;
    *s_nv = acc;
  }
  __syncthreads();
  // one thread per (group, window slot, offset)
  for (int t = threadIdx.x; t < G * nwin * APPLY_JW; t += blockDim.x) {
    const int g = t / (nwin * APPLY_JW);
    const int rem = t - g * nwin * APPLY_JW;
    const int wslot = rem / APPLY_JW;
    const int q = rem - wslot * APPLY_JW;
    if (!s_cnt[g]) continue;
    const unsigned long long u = s_union[g];
    const int a = s_lo[g] + wslot * APPLY_JW;
    if (a >= J || !((u >> a) & ((1ull << APPLY_JW) - 1))) continue;
    int v = s_base[g];
    for (int b = s_lo[g]; b < a; b += APPLY_JW)
      if ((u >> b) & ((1ull << APPLY_JW) - 1)) ++v;
    unsigned char* rec = wrec + (int64_t)v * wb;
    if (q == 0) {
      WinHead h;
      h.t = paired ? g / B + 1 : g / B;
      h.b = g % B;
      h.jlo = jmin + a;
      h.gmask = 0u;
      *reinterpret_cast<WinHead*>(rec) = h;
    }
    T* row = reinterpret_cast<T*>(rec + 16) + q * PC;
    double kv[PC_MAX];
#pragma unroll
    for (int p = 0; p < PC_MAX; ++p)
      kv[p] = (p < np && a + q < J) ? Kc[p * GJ + g * J + a + q] : 0.0;
    unsigned int m = 0;
#pragma unroll
    for (int p = 0; p < PC_MAX; ++p) {
      if (p < PC) {
        row[p] = (T)kv[p];
        if (kv[p] != 0.0) m |= 1u << ((q * NP) + (p >> 1));
      }
    }
    if (m) atomicOr(&s_gm[v], m);
  }
  __syncthreads();
  const int nv = *s_nv;
  for (int v = threadIdx.x; v < nv; v += blockDim.x)
    reinterpret_cast<WinHead*>(wrec + (int64_t)v * wb)->gmask = s_gm[v];
}

// One block per chunk of PC phases: the phases' taps K[ph][g][j] from the
// fixed-point accumulators (which are cleared for the next call), the
// per-(phase, group) bitmask of non-zero offsets, then the chunk's window
// records.  With IN_LDS the chunk's taps and masks stay in LDS; otherwise
// they go through K and mask in global memory.
template <typename T, bool IN_LDS>
__device__ __forceinline__ void finish_block(const FinishArgs& a, int chunk, unsigned char* fin_lds) {
  const int n_ph = a.n_ph, PC = a.PC, G = a.G, J = a.J, jmin = a.jmin, B = a.B, paired = a.paired,
            vg_cap = a.vg_cap;
  unsigned long long* __restrict__ Kfx = a.Kfx;
  double* __restrict__ K = a.K;
  unsigned long long* __restrict__ mask = a.mask;
  unsigned char* __restrict__ wins = a.wins;
  int* __restrict__ nvg = a.nvg;
  const int p0 = chunk * PC;
  const int np = min(PC, n_ph - p0);
  const int GJ = G * J;
  const int n = np * GJ;
  const int64_t base = (int64_t)p0 * GJ;
  double* Kc = IN_LDS ? reinterpret_cast<double*>(fin_lds) : K + base;
  unsigned long long* maskc =
      IN_LDS ? reinterpret_cast<unsigned long long*>(fin_lds + (size_t)PC * GJ * sizeof(double)) : mask + (int64_t)p0 * G;
  int* sm = reinterpret_cast<int*>(fin_lds + (IN_LDS ? (size_t)PC * (GJ + G) * sizeof(double) : 0));
  // eight accumulators per thread and round, loaded together
  for (int t0 = threadIdx.x; t0 < n; t0 += 8 * FINISH_THREADS) {
    unsigned long long v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * FINISH_THREADS;
      v[u] = t < n ? Kfx[base + t] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * FINISH_THREADS;
      if (t < n) {
        Kfx[base + t] = 0ull;
        Kc[t] = (double)(long long)v[u] * FX_INV;
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < np * G; t += blockDim.x) {
    const double* kr = Kc + (int64_t)t * J;
    unsigned long long mk = 0;
    for (int j = 0; j < J; ++j)
      if (kr[j] != 0.0) mk |= 1ull << j;
    maskc[t] = mk;
  }
  __syncthreads();
  compact_chunk<T>(chunk, n_ph, PC, G, J, jmin, B, paired, Kc, maskc, wins, nvg, vg_cap, sm);
}

template <typename T, bool IN_LDS>
__global__ void __launch_bounds__(FINISH_THREADS) k_finish(FinishArgs a) {
  extern __shared__ __align__(16) unsigned char fin_lds[];
  finish_block<T, IN_LDS>(a, blockIdx.x, fin_lds);
}

// Per phase (one thread each): every region centre rotated to the phase
// (longitude + 360 deg * phase, axis tilted by the inclination), cos(alpha),
// and the disk-cell bounding box of the caps that reach the visible
// hemisphere.  The regions and phases are read once from the caller's
// parameter block, so the weight kernel's many blocks read device memory.
// Block bid of nblk (128 threads each).
__device__ __forceinline__ void params_block(const ParamsArgs& a, int bid, int nblk) {
  const int N = a.N, n_reg = a.n_reg, max_reg = a.max_reg, n_ph = a.n_ph;
  const double incl = a.incl, diff_rot = a.diff_rot;
  const Region* __restrict__ reg = a.reg;
  const double* __restrict__ phases = a.phases;
  const int2* __restrict__ pj = a.pj;
  Region* __restrict__ reg_out = a.reg_out;
  int2* __restrict__ pj_out = a.pj_out;
  double4* __restrict__ cen = a.cen;
  int4* __restrict__ box = a.box;
  // one region list for every phase (pj == NULL): staged in LDS; per-phase
  // lists (pj[ph] = first region, count): read from the parameter block
  __shared__ Region s_reg[MAX_REGIONS];
  if (!pj)
    for (int r = threadIdx.x; r < n_reg; r += blockDim.x) s_reg[r] = reg[r];
  for (int r = bid * blockDim.x + threadIdx.x; r < n_reg; r += nblk * blockDim.x) reg_out[r] = reg[r];
  __syncthreads();
  const int ph = bid * blockDim.x + threadIdx.x;
  if (ph >= n_ph) return;
  const double phase = phases[ph];
  int2 rl = make_int2(0, n_reg);
  if (pj) {
    rl = pj[ph];
    pj_out[ph] = rl;
  }
  const Region* R = pj ? reg + rl.x : s_reg;
  // a cap point p satisfies |p - c| <= 2 sin(alpha / 2) = sqrt(2 - 2 cos
  // alpha), which bounds its projected distance from the centre
  double xlo = 2.0, xhi = -2.0, ylo = 2.0, yhi = -2.0;
  for (int r = 0; r < rl.y; ++r) {
    const Region g = R[r];
    double cx, cy, cz, rc;
    region_centre(g.lat_deg, g.lon_deg, phase, incl, diff_rot, &cx, &cy, &cz);
    {
#pragma clang fp contract(off)
      rc = sqrt(1.0 - g.radius * g.radius);
    }
    cen[(int64_t)ph * max_reg + r] = make_double4(cx, cy, cz, rc);
    const double rad = sqrt(fmax(0.0, 1.0 - rc * rc));
    if (cz <= -rad - 1e-12) continue;
    const double d = sqrt(fmax(0.0, 2.0 - 2.0 * rc)) + 1e-9;
    xlo = fmin(xlo, cx - d);
    xhi = fmax(xhi, cx + d);
    ylo = fmin(ylo, cy - d);
    yhi = fmax(yhi, cy + d);
  }
  const int i0 = (int)floor((xlo + 1.0) * 0.5 * N) - 1;
  const int i1 = (int)ceil((xhi + 1.0) * 0.5 * N) + 1;
  const int k0 = (int)floor((ylo + 1.0) * 0.5 * N) - 1;
  const int k1 = (int)ceil((yhi + 1.0) * 0.5 * N) + 1;
  box[ph] = make_int4(i0, i1, max(k0, 0), min(k1, N - 1));
}

__global__ void __launch_bounds__(128) k_params(ParamsArgs a) { params_block(a, blockIdx.x, gridDim.x); }

template <bool KAHAN32>
__device__ __forceinline__ void weights_block(const WeightsArgs& a, int ph, int slab) {
  const int N = a.N, B = a.B, J = a.J, jmin = a.jmin, G = a.G, paired = a.paired, effect = a.effect,
            n_reg_all = a.n_reg_all, max_reg = a.max_reg;
  const double u1 = a.u1, u2 = a.u2;
  const double* __restrict__ mu_b = a.mu_b;
  const int* __restrict__ col_c = a.col_c;
  const double* __restrict__ col_w = a.col_w;
  const Region* __restrict__ reg = a.reg;
  const int2* __restrict__ pj = a.pj;
  const double4* __restrict__ cen = a.cen;
  const int4* __restrict__ pbox = a.pbox;
  unsigned long long* __restrict__ Kfx = a.Kfx;
  __shared__ double rcx[MAX_REGIONS], rcy[MAX_REGIONS], rcz[MAX_REGIONS], rcos[MAX_REGIONS],
      rscal[MAX_REGIONS], rreach[MAX_REGIONS];
  __shared__ double s_mub[MAX_MU];
  __shared__ int rtype[MAX_REGIONS];
  __shared__ unsigned long long s_tab[WEIGHT_WAVES][3 * MAX_MU];  // per-wave column table

  const int nw = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int GJ = G * J;
  const double area = (2.0 / N) * (2.0 / N);

  // uniform: the slab's part of the phase's bounding box
  const int4 bx = pbox[ph];
  const int i0 = max(bx.x, slab * SLAB_COLS);
  const int i1 = min(bx.y, min(N, (slab + 1) * SLAB_COLS) - 1);
  const int k0 = bx.z, k1 = bx.w;
  if (i0 > i1 || k0 > k1) return;  // nothing of this slab is covered
  for (int b = threadIdx.x; b < B; b += blockDim.x) s_mub[b] = mu_b[b];
  // this phase's region list (uniform)
  int rbase = 0, n_reg = n_reg_all;
  if (pj) {
    const int2 rl = pj[ph];
    rbase = rl.x;
    n_reg = rl.y;
  }
  if (threadIdx.x < n_reg) {
    const double4 c4 = cen[(int64_t)ph * max_reg + threadIdx.x];
    const Region& g = reg[rbase + threadIdx.x];
    rcx[threadIdx.x] = c4.x;
    rcy[threadIdx.x] = c4.y;
    rcz[threadIdx.x] = c4.z;
    rcos[threadIdx.x] = c4.w;
    rtype[threadIdx.x] = g.type;
    rscal[threadIdx.x] = (!paired && effect != SOAP_EFFECT_BCONV) ? g.contrast : 1.0;
    // projected reach of the cap around its centre, or -1 when the cap
    // cannot reach the visible hemisphere (the bounding-box rule)
    const double rad = sqrt(fmax(0.0, 1.0 - c4.w * c4.w));
    rreach[threadIdx.x] = (c4.z <= -rad - 1e-12) ? -1.0 : sqrt(fmax(0.0, 2.0 - 2.0 * c4.w)) + 1e-9;
  }
  __syncthreads();
  unsigned long long* Kph = Kfx + (int64_t)ph * GJ;
  unsigned long long* tab = s_tab[wave];

  for (int i = i0 + wave; i <= i1; i += nw) {
    const double x = cell_coord(i, N);
    // rows of this column that any cap can reach: the hull of the chords of
    // the discs of radius reach around the projected centres
    double ylo = 2.0, yhi = -2.0;
    for (int r = 0; r < n_reg; ++r) {
      const double d = rreach[r];
      const double dx = x - rcx[r];
      if (d < 0.0 || fabs(dx) > d) continue;
      const double h = sqrt(fmax(0.0, d * d - dx * dx));
      ylo = fmin(ylo, rcy[r] - h);
      yhi = fmax(yhi, rcy[r] + h);
    }
    if (ylo > yhi) continue;  // uniform
    const int kc0 = max(k0, (int)floor((ylo + 1.0) * 0.5 * N) - 1);
    const int kc1 = min(k1, (int)ceil((yhi + 1.0) * 0.5 * N) + 1);
    const int ci = col_c[i];
    const double wi = col_w[i];
    const int ja = ci - jmin, jb = ci - 1 - jmin;
    for (int e = lane; e < G; e += 64) tab[e] = 0ull;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int kbase = kc0; kbase <= kc1; kbase += 64 * MAXC) {
      int cb[MAXC];     // bin | (type << 8), or -1 when not active
      double cw[MAXC];  // A I(mu)
      double cs[MAXC];  // owner contrast scale
#pragma unroll
      for (int q = 0; q < MAXC; ++q) {
        cb[q] = -1;
        cw[q] = 0.0;
        cs[q] = 0.0;
        const int k = kbase + lane + 64 * q;
        if (k <= kc1) {
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
              const int b = nearest_bin(mu, s_mub, B);
              const int t = rtype[own];
              cb[q] = b | (t << 8);
              cw[q] = area * limb_dark(mu, u1, u2);
              cs[q] = rscal[own];
            }
          }
        }
      }
      // Each lane sums its own cells per table row (FP32 + Kahan in the
      // FP32 mode, FP64 otherwise) and adds each sum to the wave's column
      // table as an exact fixed-point integer, so the column totals do not
      // depend on the order of the lanes.  Split tables also give every
      // active cell a removal entry (row = bin, weight -A I).
#pragma unroll
      for (int q = 0; q < MAXC; ++q) {
        if (cb[q] < 0) continue;
        const int tb = cb[q] & 0xff, tt = cb[q] >> 8;
        // active entry: first cell of this lane with this (type, bin)
        bool first = true;
#pragma unroll
        for (int q2 = 0; q2 < q; ++q2) first = first && cb[q2] != cb[q];
        if (first) {
          double part;
          if (KAHAN32) {
            float acc = 0.f, comp = 0.f;
#pragma unroll
            for (int q2 = q; q2 < MAXC; ++q2) {
              if (cb[q2] == cb[q]) {
                const float yk = (float)(cw[q2] * cs[q2]) - comp;
                const float tk = acc + yk;
                comp = (tk - acc) - yk;
                acc = tk;
              }
            }
            part = (double)acc - (double)comp;
          } else {
            double acc = 0.0;
#pragma unroll
            for (int q2 = q; q2 < MAXC; ++q2)
              if (cb[q2] == cb[q]) acc += cw[q2] * cs[q2];
            part = acc;
          }
          const int g = paired ? (tt - 1) * B + tb : tt * B + tb;
          atomicAdd(&tab[g], to_fx(part));
        }
        if (!paired) {
          // removal entry: first active cell of this lane in this bin
          bool firstb = true;
#pragma unroll
          for (int q2 = 0; q2 < q; ++q2) firstb = firstb && (cb[q2] < 0 || (cb[q2] & 0xff) != tb);
          if (firstb) {
            double part;
            if (KAHAN32) {
              float acc = 0.f, comp = 0.f;
#pragma unroll
              for (int q2 = q; q2 < MAXC; ++q2) {
                if (cb[q2] >= 0 && (cb[q2] & 0xff) == tb) {
                  const float yk = -(float)cw[q2] - comp;
                  const float tk = acc + yk;
                  comp = (tk - acc) - yk;
                  acc = tk;
                }
              }
              part = (double)acc - (double)comp;
            } else {
              double acc = 0.0;
#pragma unroll
              for (int q2 = q; q2 < MAXC; ++q2)
                if (cb[q2] >= 0 && (cb[q2] & 0xff) == tb) acc -= cw[q2];
              part = acc;
            }
            atomicAdd(&tab[tb], to_fx(part));
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // the column's sums, split onto the two integer offsets of its shift
    // (1 - w at j = c, w at j = c - 1: Eq. 11), go to the phase's table
    if (jb >= 0 && ja < J) {
      for (int e = lane; e < G; e += 64) {
        const long long v = (long long)tab[e];
        if (v == 0) continue;
        const double W = (double)v * FX_INV;
        unsigned long long* kr = Kph + e * J;
        atomicAdd(kr + ja, to_fx((1.0 - wi) * W));
        atomicAdd(kr + jb, to_fx(wi * W));
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <bool KAHAN32>
__global__ void __launch_bounds__(WEIGHT_WAVES * 64) k_weights(WeightsArgs a) {
  const int ph = blockIdx.x / a.n_slabs;
  weights_block<KAHAN32>(a, ph, blockIdx.x - ph * a.n_slabs);
}

// Differential rotation: the cells of one column no longer share a shift, so
// every active cell splits its weight A I (times the owner's scale in split
// tables) onto its own two offsets (Eq. 11) in a per-wave LDS table
// [G][J] of exact 64-bit fixed-point sums (the removal rows of split tables
// likewise), which the wave adds to the phase's tap table once it has walked
// all its columns.  Ownership, bins and the rows each column can reach are
// decided as in k_weights.  Per-cell weights are products in double in both
// precisions; the fixed-point sums are exact, so the totals do not depend
// on the order of cells, lanes or columns.
__global__ void __launch_bounds__(WEIGHT_WAVES * 64) k_weights_dr(
    int N, int B, int J, int jmin, int G, int paired, int n_slabs, double u1, double u2, int effect, double vsini,
    double diff_rot, double sin_i, double cos_i, double dln, const double* __restrict__ mu_b,
    const Region* __restrict__ reg, int n_reg_all, int max_reg, const int2* __restrict__ pj,
    const double4* __restrict__ cen, const int4* __restrict__ pbox, unsigned long long* __restrict__ Kfx) {
  __shared__ double rcx[MAX_REGIONS], rcy[MAX_REGIONS], rcz[MAX_REGIONS], rcos[MAX_REGIONS],
      rscal[MAX_REGIONS], rreach[MAX_REGIONS];
  __shared__ double s_mub[MAX_MU];
  __shared__ int rtype[MAX_REGIONS];
  extern __shared__ unsigned long long s_drtab[];  // [WEIGHT_WAVES][G * J]

  const int ph = blockIdx.x / n_slabs;
  const int slab = blockIdx.x - ph * n_slabs;
  const int nw = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int GJ = G * J;
  const double area = (2.0 / N) * (2.0 / N);

  const int4 bx = pbox[ph];
  const int i0 = max(bx.x, slab * SLAB_COLS);
  const int i1 = min(bx.y, min(N, (slab + 1) * SLAB_COLS) - 1);
  const int k0 = bx.z, k1 = bx.w;
  if (i0 > i1 || k0 > k1) return;  // nothing of this slab is covered
  for (int b = threadIdx.x; b < B; b += blockDim.x) s_mub[b] = mu_b[b];
  int rbase = 0, n_reg = n_reg_all;
  if (pj) {
    const int2 rl = pj[ph];
    rbase = rl.x;
    n_reg = rl.y;
  }
  if (threadIdx.x < n_reg) {
    const double4 c4 = cen[(int64_t)ph * max_reg + threadIdx.x];
    const Region& g = reg[rbase + threadIdx.x];
    rcx[threadIdx.x] = c4.x;
    rcy[threadIdx.x] = c4.y;
    rcz[threadIdx.x] = c4.z;
    rcos[threadIdx.x] = c4.w;
    rtype[threadIdx.x] = g.type;
    rscal[threadIdx.x] = (!paired && effect != SOAP_EFFECT_BCONV) ? g.contrast : 1.0;
    const double rad = sqrt(fmax(0.0, 1.0 - c4.w * c4.w));
    rreach[threadIdx.x] = (c4.z <= -rad - 1e-12) ? -1.0 : sqrt(fmax(0.0, 2.0 - 2.0 * c4.w)) + 1e-9;
  }
  unsigned long long* tab = s_drtab + (size_t)wave * GJ;
  for (int e = lane; e < GJ; e += 64) tab[e] = 0ull;
  __syncthreads();

  for (int i = i0 + wave; i <= i1; i += nw) {
    const double x = cell_coord(i, N);
    double ylo = 2.0, yhi = -2.0;
    for (int r = 0; r < n_reg; ++r) {
      const double d = rreach[r];
      const double dx = x - rcx[r];
      if (d < 0.0 || fabs(dx) > d) continue;
      const double h = sqrt(fmax(0.0, d * d - dx * dx));
      ylo = fmin(ylo, rcy[r] - h);
      yhi = fmax(yhi, rcy[r] + h);
    }
    if (ylo > yhi) continue;  // uniform
    const int kc0 = max(k0, (int)floor((ylo + 1.0) * 0.5 * N) - 1);
    const int kc1 = min(k1, (int)ceil((yhi + 1.0) * 0.5 * N) + 1);
    for (int k = kc0 + lane; k <= kc1; k += 64) {
      const double y = cell_coord(k, N);
      double r2;
      {
#pragma clang fp contract(off)
        r2 = x * x + y * y;
      }
      if (!(r2 < 1.0)) continue;
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
      if (own < 0) continue;
      const int b = nearest_bin(mu, s_mub, B);
      const int t = rtype[own];
      int cc;
      double w;
      cell_shift(x, y, mu, vsini, diff_rot, sin_i, cos_i, dln, &cc, &w);
      const int ja = cc - jmin, jb = cc - 1 - jmin;
      if (jb < 0 || ja >= J) continue;  // unreachable: the offset range bounds every shift
      const double aw = area * limb_dark(mu, u1, u2);
      const int g = paired ? (t - 1) * B + b : t * B + b;
      const double W = aw * rscal[own];
      atomicAdd(&tab[g * J + ja], to_fx((1.0 - w) * W));
      atomicAdd(&tab[g * J + jb], to_fx(w * W));
      if (!paired) {
        // removal entry (row = bin, weight -A I)
        atomicAdd(&tab[b * J + ja], to_fx(-(1.0 - w) * aw));
        atomicAdd(&tab[b * J + jb], to_fx(-w * aw));
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  unsigned long long* Kph = Kfx + (int64_t)ph * GJ;
  for (int e = lane; e < GJ; e += 64) {
    const unsigned long long v = tab[e];
    if (v) atomicAdd(Kph + e, v);
  }
}

namespace {

ParamsArgs params_args(const soap_ctx* c, const Plan& pl, const Region* d_reg, int n_reg, int max_reg,
                       const double* d_ph, const int2* d_pj, const WeightsOut& o) {
  return ParamsArgs{c->N, n_reg, max_reg, pl.n_ph, c->incl, c->diff_rot, d_reg, d_ph, d_pj, o.reg, o.pj, o.cen, o.box};
}

WeightsArgs weights_args(const soap_ctx* c, const Plan& pl, int n_reg, int max_reg, const int2* pj,
                         const WeightsOut& o) {
  return WeightsArgs{c->N,     c->B,  c->J,       c->jmin,    pl.G,      pl.paired, pl.n_slabs,
                     pl.effect, n_reg, max_reg,   c->u1,      c->u2,     c->d_mu,   c->d_col_c,
                     c->d_col_w, o.reg, pj,       o.cen,      o.box,     o.Kfx};
}

FinishArgs finish_args(const soap_ctx* c, const Plan& pl, const WeightsOut& o) {
  return FinishArgs{pl.n_ph, pl.pc, pl.G, c->J, c->jmin, c->B, pl.paired, pl.vg_cap, o.Kfx, o.K, o.mask, o.wins,
                    o.nvg};
}

// dynamic LDS of the finish kernel and whether the chunk's taps fit in it;
// false when even the compaction scratch does not fit
bool finish_lds(const soap_ctx* c, const Plan& pl, size_t* lds, bool* in_lds) {
  const size_t cmp = (size_t)(6 * pl.G + pl.vg_cap + 2) * sizeof(int);
  const size_t tab = (size_t)pl.pc * ((size_t)pl.G * c->J + pl.G) * sizeof(double);
  *in_lds = tab + cmp <= 60 * 1024;
  *lds = *in_lds ? tab + cmp : cmp;
  return *lds <= 60 * 1024;
}

__device__ __forceinline__ int find_cfg(const int* __restrict__ off, int n, int b) {
  int lo = 0, hi = n;  // last configuration with off[cfg] <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

}  // namespace

// Work-list forms: configuration i owns blocks off[i] .. off[i + 1] - 1.
__global__ void __launch_bounds__(128) k_params_batch(const ParamsArgs* __restrict__ args, const int* __restrict__ off,
                                                      int n) {
  const int i = find_cfg(off, n, blockIdx.x);
  const ParamsArgs a = args[i];
  params_block(a, blockIdx.x - off[i], off[i + 1] - off[i]);
}

// one block per listed (configuration, phase, slab): blk[b] = (cfg, ph, slab)
template <bool KAHAN32>
__global__ void __launch_bounds__(WEIGHT_WAVES * 64) k_weights_batch(const WeightsArgs* __restrict__ args,
                                                                     const int4* __restrict__ blk) {
  const int4 t = blk[blockIdx.x];
  const WeightsArgs a = args[t.x];
  weights_block<KAHAN32>(a, t.y, t.z);
}

template <typename T, bool IN_LDS>
__global__ void __launch_bounds__(FINISH_THREADS) k_finish_batch(const FinishArgs* __restrict__ args,
                                                                 const int* __restrict__ off, int n) {
  extern __shared__ __align__(16) unsigned char fin_lds[];
  const int i = find_cfg(off, n, blockIdx.x);
  const FinishArgs a = args[i];
  finish_block<T, IN_LDS>(a, blockIdx.x - off[i], fin_lds);
}

hipError_t launch_weights(soap_ctx* c, const Plan& pl, const Region* d_reg, int n_reg, int max_reg,
                          const double* d_ph, const int2* d_pj, const WeightsOut& o, hipStream_t st) {
  hipLaunchKernelGGL(k_params, dim3((unsigned)((pl.n_ph + 127) / 128)), dim3(128), 0, st,
                     params_args(c, pl, d_reg, n_reg, max_reg, d_ph, d_pj, o));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int2* pj = d_pj ? o.pj : nullptr;
  dim3 grid((unsigned)pl.n_slabs * (unsigned)pl.n_ph);
  if (c->diff_rot != 0.0) {
    const size_t lds = (size_t)WEIGHT_WAVES * pl.G * c->J * sizeof(unsigned long long);
    if (pl.G * c->J > DR_TAB_MAX) return hipErrorInvalidValue;  // refused at init
    hipLaunchKernelGGL(k_weights_dr, grid, dim3(64 * WEIGHT_WAVES), lds, st, c->N, c->B, c->J, c->jmin, pl.G,
                       pl.paired, pl.n_slabs, c->u1, c->u2, pl.effect, c->vsini, c->diff_rot, c->sin_i, c->cos_i,
                       c->dln, c->d_mu, o.reg, n_reg, max_reg, pj, o.cen, o.box, o.Kfx);
    return hipGetLastError();
  }
  const WeightsArgs wa = weights_args(c, pl, n_reg, max_reg, pj, o);
  if (c->prec == SOAP_PREC_FP32)
    hipLaunchKernelGGL(k_weights<true>, grid, dim3(64 * WEIGHT_WAVES), 0, st, wa);
  else
    hipLaunchKernelGGL(k_weights<false>, grid, dim3(64 * WEIGHT_WAVES), 0, st, wa);
  return hipGetLastError();
}

hipError_t launch_finish(soap_ctx* c, const Plan& pl, const WeightsOut& o, hipStream_t st) {
  if (!pc_valid(c->prec == SOAP_PREC_FP32, pl.pc)) return hipErrorInvalidValue;
  size_t lds = 0;
  bool in_lds = false;
  if (!finish_lds(c, pl, &lds, &in_lds)) return hipErrorInvalidValue;
  const dim3 grid(pl.n_chunks), block(FINISH_THREADS);
  const FinishArgs fa = finish_args(c, pl, o);
  if (c->prec == SOAP_PREC_FP32) {
    if (in_lds)
      hipLaunchKernelGGL((k_finish<float, true>), grid, block, lds, st, fa);
    else
      hipLaunchKernelGGL((k_finish<float, false>), grid, block, lds, st, fa);
  } else {
    if (in_lds)
      hipLaunchKernelGGL((k_finish<double, true>), grid, block, lds, st, fa);
    else
      hipLaunchKernelGGL((k_finish<double, false>), grid, block, lds, st, fa);
  }
  return hipGetLastError();
}

// ---- table kernels of many configurations ----------------------------------

namespace {

size_t al256(size_t b) { return 256 * ((b + 255) / 256); }

// one launch's argument array and block offsets, appended to the buffer
template <typename A>
hipError_t upload_launch(const std::vector<A>& args, const std::vector<int>& blocks, unsigned char* base,
                         size_t* used, TableBatch::Launch* L) {
  L->n_cfg = (int)args.size();
  L->n_blocks = 0;
  if (args.empty()) return hipSuccess;
  std::vector<int> off(args.size() + 1, 0);
  for (size_t i = 0; i < args.size(); ++i) off[i + 1] = off[i] + blocks[i];
  L->n_blocks = off.back();
  L->args = base + *used;
  *used += al256(sizeof(A) * args.size());
  L->off = reinterpret_cast<int*>(base + *used);
  *used += al256(sizeof(int) * off.size());
  hipError_t e = hipMemcpy(L->args, args.data(), sizeof(A) * args.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemcpy(L->off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice);
}

}  // namespace

// Slabs of disk columns that the visible caps of a configuration can reach
// at one phase, from the region centres computed on the host with the
// kernels' formulas and widened by one slab on each side (so host/device
// rounding cannot drop a column; the kernel applies the exact bounds).
void reachable_slabs(const TableBatchCfg& q, int ph, std::vector<int4>& out, int cfg) {
#ifndef __HIP_DEVICE_COMPILE__  // host code (region_centre is host-callable in the host pass only)
  const soap_ctx* c = q.c;
  double xlo = 2.0, xhi = -2.0;
  for (int r = 0; r < q.n_reg; ++r) {
    const Region& g = q.h_reg[r];
    double cx, cy, cz;
    region_centre(g.lat_deg, g.lon_deg, q.h_ph[ph], c->incl, c->diff_rot, &cx, &cy, &cz);
    const double rc = std::sqrt(1.0 - g.radius * g.radius);
    const double rad = std::sqrt(std::fmax(0.0, 1.0 - rc * rc));
    if (cz <= -rad - 1e-6) continue;  // the kernels drop it below -rad - 1e-12
    const double d = std::sqrt(std::fmax(0.0, 2.0 - 2.0 * rc)) + 1e-6;
    xlo = std::fmin(xlo, cx - d);
    xhi = std::fmax(xhi, cx + d);
  }
  if (xlo > xhi) return;
  const int N = c->N;
  const int i0 = std::max(0, (int)std::floor((xlo + 1.0) * 0.5 * N) - 2);
  const int i1 = std::min(N - 1, (int)std::ceil((xhi + 1.0) * 0.5 * N) + 2);
  if (i0 > i1) return;
  const int s0 = std::max(0, i0 / SLAB_COLS - 1), s1 = std::min(q.pl.n_slabs - 1, i1 / SLAB_COLS + 1);
  for (int sl = s0; sl <= s1; ++sl) out.push_back(make_int4(cfg, ph, sl, 0));
#endif
}

size_t table_batch_bytes(const TableBatchCfg* cfgs, int n) {
  size_t blocks = 0;
  for (int i = 0; i < n; ++i) blocks += (size_t)cfgs[i].pl.n_ph * cfgs[i].pl.n_slabs;  // upper bound
  // every configuration appears in params, one weights list and one finish list
  return al256(sizeof(ParamsArgs) * n) + al256(sizeof(WeightsArgs) * n) * 2 + al256(sizeof(FinishArgs) * n) * 4 +
         5 * al256(sizeof(int) * (n + 1)) + 2 * al256(sizeof(int4) * blocks);
}

hipError_t table_batch_upload(const TableBatchCfg* cfgs, int n, void* d_buf, TableBatch* tb) {
  std::vector<ParamsArgs> pa;
  std::vector<int> pb;
  std::vector<WeightsArgs> wa[2];
  std::vector<int4> wblk[2];
  std::vector<FinishArgs> fa[4];
  std::vector<int> fb[4];
  size_t flds[4] = {0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    const TableBatchCfg& q = cfgs[i];
    const soap_ctx* c = q.c;
    if (c->diff_rot != 0.0 || !pc_valid(c->prec == SOAP_PREC_FP32, q.pl.pc)) return hipErrorInvalidValue;
    pa.push_back(params_args(c, q.pl, q.d_reg, q.n_reg, q.max_reg, q.d_ph, nullptr, q.o));
    pb.push_back((q.pl.n_ph + 127) / 128);
    const int w = c->prec == SOAP_PREC_FP32 ? 0 : 1;
    const int wi = (int)wa[w].size();
    wa[w].push_back(weights_args(c, q.pl, q.n_reg, q.max_reg, nullptr, q.o));
    for (int ph = 0; ph < q.pl.n_ph; ++ph) reachable_slabs(q, ph, wblk[w], wi);
    size_t lds = 0;
    bool in_lds = false;
    if (!finish_lds(c, q.pl, &lds, &in_lds)) return hipErrorInvalidValue;
    const int f = 2 * w + (in_lds ? 0 : 1);
    fa[f].push_back(finish_args(c, q.pl, q.o));
    fb[f].push_back(q.pl.n_chunks);
    flds[f] = std::max(flds[f], lds);
  }
  unsigned char* base = static_cast<unsigned char*>(d_buf);
  size_t used = 0;
  hipError_t e = upload_launch(pa, pb, base, &used, &tb->params);
  for (int w = 0; w < 2 && e == hipSuccess; ++w) {
    TableBatch::Launch& L = tb->weights[w];
    L.n_cfg = (int)wa[w].size();
    L.n_blocks = (int)wblk[w].size();
    if (wa[w].empty() || wblk[w].empty()) {
      L.n_blocks = 0;
      continue;
    }
    L.args = base + used;
    used += al256(sizeof(WeightsArgs) * wa[w].size());
    L.blk = reinterpret_cast<int4*>(base + used);
    used += al256(sizeof(int4) * wblk[w].size());
    e = hipMemcpy(L.args, wa[w].data(), sizeof(WeightsArgs) * wa[w].size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(L.blk, wblk[w].data(), sizeof(int4) * wblk[w].size(), hipMemcpyHostToDevice);
  }
  for (int f = 0; f < 4 && e == hipSuccess; ++f) {
    e = upload_launch(fa[f], fb[f], base, &used, &tb->finish[f]);
    tb->finish[f].lds = flds[f];
  }
  return e;
}

hipError_t table_batch_launch(const TableBatch& tb, hipStream_t st) {
  if (tb.params.n_blocks > 0)
    hipLaunchKernelGGL(k_params_batch, dim3((unsigned)tb.params.n_blocks), dim3(128), 0, st,
                       static_cast<const ParamsArgs*>(tb.params.args), tb.params.off, tb.params.n_cfg);
  const dim3 wblock(64 * WEIGHT_WAVES), fblock(FINISH_THREADS);
  const TableBatch::Launch* W = tb.weights;
  if (W[0].n_blocks > 0)
    hipLaunchKernelGGL(k_weights_batch<true>, dim3((unsigned)W[0].n_blocks), wblock, 0, st,
                       static_cast<const WeightsArgs*>(W[0].args), W[0].blk);
  if (W[1].n_blocks > 0)
    hipLaunchKernelGGL(k_weights_batch<false>, dim3((unsigned)W[1].n_blocks), wblock, 0, st,
                       static_cast<const WeightsArgs*>(W[1].args), W[1].blk);
  const TableBatch::Launch* F = tb.finish;
  if (F[0].n_blocks > 0)
    hipLaunchKernelGGL((k_finish_batch<float, true>), dim3((unsigned)F[0].n_blocks), fblock, F[0].lds, st,
                       static_cast<const FinishArgs*>(F[0].args), F[0].off, F[0].n_cfg);
  if (F[1].n_blocks > 0)
    hipLaunchKernelGGL((k_finish_batch<float, false>), dim3((unsigned)F[1].n_blocks), fblock, F[1].lds, st,
                       static_cast<const FinishArgs*>(F[1].args), F[1].off, F[1].n_cfg);
  if (F[2].n_blocks > 0)
    hipLaunchKernelGGL((k_finish_batch<double, true>), dim3((unsigned)F[2].n_blocks), fblock, F[2].lds, st,
                       static_cast<const FinishArgs*>(F[2].args), F[2].off, F[2].n_cfg);
  if (F[3].n_blocks > 0)
    hipLaunchKernelGGL((k_finish_batch<double, false>), dim3((unsigned)F[3].n_blocks), fblock, F[3].lds, st,
                       static_cast<const FinishArgs*>(F[3].args), F[3].off, F[3].n_cfg);
  return hipGetLastError();
}

}  // namespace soap
