// Final spectra of a chunk of phases over a tile of pixels (section 3.3,
// Algorithm 5 with Eqs. 1-4).
//
// With the quiet integrated spectrum Q resident, Eq. 4 gives each phase's
// spectrum as Q minus the summed per-cell differences of the active cells.
// Grouped by disk column and collapsed onto integer pixel offsets (see
// weights.hip):
//
//   paired tables (one row per active type and mu bin b):
//     F[p][m] = Q[m] + sum_{t,b,j} K[p][t,b][j] * (A_{t,b}(m, j) - S_{q,b}[m - j])
//   with A = C_{t,b}[m] S_{t,b}[m - j]  (Eq. 3, total effect),
//            C_{t,b}[m] S_{q,b}[m - j]  (Eq. 1, flux effect),
//            S_{t,b}[m - j]             (Eq. 2, convective effect);
//   split tables (scalar contrasts other than one): quiet-removal rows with
//   negative taps on S_{q,b} and active rows with contrast-scaled taps on A.
// The contrast multiplies after the shift, at the output pixel m.
//
// Work split: one block = 256 threads x APPLY_R consecutive pixels (one tile)
// x one chunk of PC phases.  The PC x APPLY_R accumulators live in registers.
// For each window of APPLY_JW offsets of one group, every thread loads its
// 11-sample source windows with three aligned 16-byte loads from the row copy
// whose shift matches the window start (rows are padded with their end
// samples, so no load needs a bounds check and the end-value hold of the
// interpolation is built in).  Then, offset by offset, the chunk's taps for
// that offset are read into scalar registers and every phase with a tap
// there adds it with fused multiply-adds; a wave-uniform bit test skips
// phases without one, so only non-zero taps cost arithmetic.  The next
// window's loads are issued before the current one is consumed.  The
// block-to-work mapping keeps the chunks of one tile on one XCD so their
// shared input windows hit the same L2.  The final combine adds Q in double.
#include "soap_internal.hpp"

namespace soap {

namespace {

// 12 consecutive elements from an aligned address (the 11-sample window of
// APPLY_R + APPLY_JW - 1 values plus one)
template <typename T>
struct Win12 {
  T v[12];
};

template <typename T>
__device__ __forceinline__ void load12(Win12<T>& w, const T* p) {
  if constexpr (sizeof(T) == 4) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float4 f = q[k];
      w.v[4 * k + 0] = f.x;
      w.v[4 * k + 1] = f.y;
      w.v[4 * k + 2] = f.z;
      w.v[4 * k + 3] = f.w;
    }
  } else {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double2 f = q[k];
      w.v[2 * k + 0] = f.x;
      w.v[2 * k + 1] = f.y;
    }
  }
}

template <typename T>
__device__ __forceinline__ void load4(T (&c)[4], const T* p) {
  if constexpr (sizeof(T) == 4) {
    float4 f = *reinterpret_cast<const float4*>(p);
    c[0] = f.x;
    c[1] = f.y;
    c[2] = f.z;
    c[3] = f.w;
  } else {
    double2 a = reinterpret_cast<const double2*>(p)[0];
    double2 b = reinterpret_cast<const double2*>(p)[1];
    c[0] = a.x;
    c[1] = a.y;
    c[2] = b.x;
    c[3] = b.y;
  }
}

// operands of one window: D[q][r] = Ca[r] * A[m_r - j] - B[m_r - j],
// j = jlo + q, with window sample s = r - q + APPLY_JW - 1
template <typename T>
struct Operands {
  Win12<T> a, b;
  T c[4];
  int sub;  // 1: D = C A - B, 0: D = C A
};

template <typename T>
struct ApplyArgs {
  int64_t P, Pstride;
  int B, n_ph, n_chunks, n_tiles, effect, paired, vg_cap, vec_ok;
  const T *Sq, *Ss, *Sf, *Cs, *Cf;
  const double* Q;
  const VGroup* vgs;
  const int* nvg;
  const T* taps;
  T* out;
};

template <typename T, int R, int JW>
__device__ __forceinline__ void fetch(Operands<T>& o, const ApplyArgs<T>& A, int g, int jlo, int64_t m0) {
  // group -> (type, bin) and the effect's operands
  int t, b;
  if (A.paired) {
    t = g / A.B + 1;
    b = g - (t - 1) * A.B;
  } else {
    t = g / A.B;
    b = g - t * A.B;
  }
  const int64_t rs = (int64_t)NCOPY * A.Pstride;  // stride between mu-bin rows
  const T* sq = A.Sq + (int64_t)b * rs;
  const T* src;
  const T* con = nullptr;
  const T* sub = nullptr;
  if (t == 0) {
    src = sq;
  } else {
    const T* ct = nullptr;
    if (A.Cs) ct = (t == SOAP_SPOT) ? A.Cs : A.Cf + (int64_t)b * A.Pstride;
    if (A.effect == SOAP_EFFECT_FLUX) {
      src = sq;
      con = ct;
    } else {
      src = (t == SOAP_SPOT ? A.Ss : A.Sf) + (int64_t)b * rs;
      con = (A.effect == SOAP_EFFECT_TOT) ? ct : nullptr;
    }
    if (A.paired) sub = sq;
  }
  // window start m0 - jlo - (JW - 1): an aligned load from the row copy
  // shifted by the start's distance d from alignment
  const int off = -jlo - (JW - 1);
  const int d = off & 3;
  const int64_t at = (int64_t)d * A.Pstride + m0 + (off - d);
  load12(o.a, src + at);
  o.sub = sub ? 1 : 0;
  if (sub && sub != src) load12(o.b, sub + at);
  else if (sub) o.b = o.a;
  if (con) {
    load4(o.c, con + m0);
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) o.c[r] = T(1);
  }
}

// One window: for every offset q with any tap in the chunk, form the
// difference row, read the chunk's PC taps of that offset into scalar
// registers, and let every phase with a tap add k * D with fused
// multiply-adds (a wave-uniform bit test skips the others).
template <typename T, int R, int PC, int JW>
__device__ __forceinline__ void consume(T (&acc)[PC][R], const Operands<T>& o, const VGroup& vg, const T* tw) {
  unsigned m[JW];
#pragma unroll
  for (int q = 0; q < JW; ++q) m[q] = vg.qmask[q];
#pragma unroll
  for (int q = 0; q < JW; ++q) {
    if (m[q] == 0) continue;
    T D[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = r - q + JW - 1;
      D[r] = o.sub ? fma(o.c[r], o.a.v[s], -o.b.v[s]) : o.c[r] * o.a.v[s];
    }
    const T* kq = tw + q * PC_MAX;
    T k[PC];
#pragma unroll
    for (int p = 0; p < PC; ++p) k[p] = kq[p];
#pragma unroll
    for (int p = 0; p < PC; ++p) {
      if ((m[q] >> p) & 1u) {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[p][r] = fma(k[p], D[r], acc[p][r]);
      }
    }
  }
}

}  // namespace

template <typename T, int R, int PC, int JW>
__global__ void __launch_bounds__(APPLY_THREADS) k_apply(ApplyArgs<T> A) {
  static_assert(R == 4 && JW == 8, "window loads are written for 4 pixels x 8 offsets");
  const int total = A.n_tiles * A.n_chunks;
  const int per_xcd = (total + 7) / 8;
  const int bid = blockIdx.x;
  const int w = (bid & 7) * per_xcd + (bid >> 3);
  if (w >= total) return;
  const int tile = w / A.n_chunks;
  const int chunk = w - tile * A.n_chunks;
  const int64_t m0 = (int64_t)tile * (R * APPLY_THREADS) + (int64_t)threadIdx.x * R;

  T acc[PC][R];
#pragma unroll
  for (int p = 0; p < PC; ++p)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[p][r] = T(0);

  const int nv = A.nvg[chunk];
  const VGroup* vg = A.vgs + (int64_t)chunk * A.vg_cap;
  const T* tw = A.taps + (int64_t)chunk * A.vg_cap * JW * PC_MAX;
  Operands<T> o0, o1;
  if (nv > 0) fetch<T, R, JW>(o0, A, vg[0].g, vg[0].jlo, m0);
  for (int v = 0; v < nv; v += 2) {
    if (v + 1 < nv) fetch<T, R, JW>(o1, A, vg[v + 1].g, vg[v + 1].jlo, m0);
    consume<T, R, PC, JW>(acc, o0, vg[v], tw + (int64_t)v * JW * PC_MAX);
    if (v + 1 < nv) {
      if (v + 2 < nv) fetch<T, R, JW>(o0, A, vg[v + 2].g, vg[v + 2].jlo, m0);
      consume<T, R, PC, JW>(acc, o1, vg[v + 1], tw + (int64_t)(v + 1) * JW * PC_MAX);
    }
  }

  double Qr[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Qr[r] = A.Q[m0 + r];  // Q is padded to whole tiles
  const int p0 = chunk * PC;
  const bool full = A.vec_ok && (m0 + R <= A.P);
#pragma unroll
  for (int p = 0; p < PC; ++p) {
    if (p0 + p >= A.n_ph) break;
    T* row = A.out + (int64_t)(p0 + p) * A.P;
    T vals[R];
#pragma unroll
    for (int r = 0; r < R; ++r) vals[r] = (T)(Qr[r] + (double)acc[p][r]);
    if (full) {
      if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(row + m0) = make_float4(vals[0], vals[1], vals[2], vals[3]);
      } else {
        reinterpret_cast<double2*>(row + m0)[0] = make_double2(vals[0], vals[1]);
        reinterpret_cast<double2*>(row + m0)[1] = make_double2(vals[2], vals[3]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (m0 + r < A.P) row[m0 + r] = vals[r];
    }
  }
}

hipError_t launch_apply(soap_ctx* c, const Plan& pl, const VGroup* d_vg, const int* d_nvg, const void* d_taps,
                        void* d_flux) {
  const int total = pl.n_chunks * c->n_tiles;
  const int per_xcd = (total + 7) / 8;
  dim3 grid(8 * per_xcd);
  const bool vec_ok = (c->P % APPLY_R == 0) &&
                      (reinterpret_cast<uintptr_t>(d_flux) % (APPLY_R * c->esize) == 0);
  if (c->prec == SOAP_PREC_FP32) {
    ApplyArgs<float> A{c->P, c->Pstride, c->B, pl.n_ph, pl.n_chunks, c->n_tiles, pl.effect, pl.paired, pl.vg_cap,
                       vec_ok ? 1 : 0,
                       (const float*)c->d_spec[0], (const float*)c->d_spec[1], (const float*)c->d_spec[2],
                       (const float*)c->d_con_spot, (const float*)c->d_con_fac, c->d_Q, d_vg, d_nvg,
                       (const float*)d_taps, (float*)d_flux};
    hipLaunchKernelGGL((k_apply<float, APPLY_R, PC_F32, APPLY_JW>), grid, dim3(APPLY_THREADS), 0, c->stream, A);
  } else {
    ApplyArgs<double> A{c->P, c->Pstride, c->B, pl.n_ph, pl.n_chunks, c->n_tiles, pl.effect, pl.paired,
                        pl.vg_cap, vec_ok ? 1 : 0,
                        (const double*)c->d_spec[0], (const double*)c->d_spec[1], (const double*)c->d_spec[2],
                        (const double*)c->d_con_spot, (const double*)c->d_con_fac, c->d_Q, d_vg, d_nvg,
                        (const double*)d_taps, (double*)d_flux};
    hipLaunchKernelGGL((k_apply<double, APPLY_R, PC_F64, APPLY_JW>), grid, dim3(APPLY_THREADS), 0, c->stream, A);
  }
  return hipGetLastError();
}

}  // namespace soap
