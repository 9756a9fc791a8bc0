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
// source windows with aligned 16-byte loads (rows are padded with their end
// samples, so no load needs a bounds check and the end-value hold of the
// interpolation is built in), forms the APPLY_JW x APPLY_R differences once,
// and every phase of the chunk applies its runs of <= 4 taps to them with
// fused multiply-adds, dispatched on a wave-uniform code.  The next window's
// loads are issued before the current one is consumed.  The block-to-work
// mapping keeps the chunks of one tile on one XCD so their shared input
// windows hit the same L2.  The final combine adds Q in double.
#include "soap_internal.hpp"

namespace soap {

namespace {

template <int Q0, int W, typename T, int R, int JW>
__device__ __forceinline__ void run_taps(T (&a)[R], const T (&D)[JW][R], const T* k) {
  if constexpr (Q0 + W <= JW) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T s = a[r];
#pragma unroll
      for (int q = 0; q < W; ++q) s = fma(k[q], D[Q0 + q][r], s);
      a[r] = s;
    }
  }
}

template <typename T, int R, int JW>
__device__ __forceinline__ void apply_entry(T (&a)[R], const T (&D)[JW][R], int code, const T* k) {
  static_assert(JW == 8, "dispatch table is written for 8-offset windows");
#define SOAP_CASE(Q0, W) \
  case Q0 * 4 + (W - 1): \
    run_taps<Q0, W, T, R, JW>(a, D, k); \
    break;
#define SOAP_CASES(Q0) SOAP_CASE(Q0, 1) SOAP_CASE(Q0, 2) SOAP_CASE(Q0, 3) SOAP_CASE(Q0, 4)
  switch (code) {
    SOAP_CASES(0)
    SOAP_CASES(1)
    SOAP_CASES(2)
    SOAP_CASES(3)
    SOAP_CASES(4)
    SOAP_CASES(5)
    SOAP_CASES(6)
    SOAP_CASES(7)
    default:
      break;
  }
#undef SOAP_CASES
#undef SOAP_CASE
}

// 16 consecutive elements starting at an aligned address
template <typename T>
struct Win16 {
  T v[16];
};

template <typename T>
__device__ __forceinline__ void load16(Win16<T>& w, const T* p) {
  if constexpr (sizeof(T) == 4) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float4 f = q[k];
      w.v[4 * k + 0] = f.x;
      w.v[4 * k + 1] = f.y;
      w.v[4 * k + 2] = f.z;
      w.v[4 * k + 3] = f.w;
    }
  } else {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
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
// j = jlo + q, A / B / Ca optional
template <typename T>
struct Operands {
  Win16<T> a, b;
  T c[4];
  int d;        // offset of the window start inside the aligned loads
  int kind;     // bit 0: contrast, bit 1: subtract B, bit 2: B is A
};

template <typename T>
struct ApplyArgs {
  int64_t P, Pstride;
  int B, n_ph, n_chunks, n_tiles, effect, paired, vg_cap, vec_ok;
  const T *Sq, *Ss, *Sf, *Cs, *Cf;
  const double* Q;
  const VGroup* vgs;
  const int* nvg;
  const Entry<T>* ents;
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
  const T* sq = A.Sq + (int64_t)b * A.Pstride;
  const T* src;
  const T* con = nullptr;
  const T* sub = nullptr;
  if (t == 0) {
    src = sq;
  } else {
    const T* st = (t == SOAP_SPOT ? A.Ss : A.Sf);
    const T* ct = nullptr;
    if (A.Cs) ct = (t == SOAP_SPOT) ? A.Cs : A.Cf + (int64_t)b * A.Pstride;
    if (A.effect == SOAP_EFFECT_FLUX) {
      src = sq;
      con = ct;
    } else {
      src = st + (int64_t)b * A.Pstride;
      con = (A.effect == SOAP_EFFECT_TOT) ? ct : nullptr;
    }
    if (A.paired) sub = sq;
  }
  // window start m0 - jlo - (JW - 1); aligned base and the offset inside it
  const int off = -jlo - (JW - 1);
  o.d = off & 3;
  const int64_t base = m0 + (off - o.d);
  o.kind = (con ? 1 : 0) | (sub ? 2 : 0) | ((sub && sub == src) ? 4 : 0);
  load16(o.a, src + base);
  if (sub && sub != src) load16(o.b, sub + base);
  if (con) load4(o.c, con + m0);
}

template <typename T, int R, int JW, int DD, int KIND>
__device__ __forceinline__ void form_d(T (&D)[JW][R], const Operands<T>& o) {
#pragma unroll
  for (int q = 0; q < JW; ++q)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = r - q + JW - 1 + DD;
      const T av = o.a.v[s];
      if constexpr (KIND == 0) D[q][r] = av;
      if constexpr (KIND == 1) D[q][r] = o.c[r] * av;
      if constexpr (KIND == 2) D[q][r] = av - o.b.v[s];
      if constexpr (KIND == 3) D[q][r] = fma(o.c[r], av, -o.b.v[s]);
      if constexpr (KIND == 6) D[q][r] = T(0);  // (1 - 1) * S: flux effect at unit contrast
      if constexpr (KIND == 7) D[q][r] = fma(o.c[r], av, -av);
    }
}

template <typename T, int R, int JW, int DD>
__device__ __forceinline__ void form_kind(T (&D)[JW][R], const Operands<T>& o) {
  switch (o.kind) {
    case 0: form_d<T, R, JW, DD, 0>(D, o); break;
    case 1: form_d<T, R, JW, DD, 1>(D, o); break;
    case 2: form_d<T, R, JW, DD, 2>(D, o); break;
    case 3: form_d<T, R, JW, DD, 3>(D, o); break;
    case 6: form_d<T, R, JW, DD, 6>(D, o); break;
    case 7: form_d<T, R, JW, DD, 7>(D, o); break;
    default: break;
  }
}

template <typename T, int R, int JW>
__device__ __forceinline__ void form(T (&D)[JW][R], const Operands<T>& o) {
  switch (o.d) {
    case 0: form_kind<T, R, JW, 0>(D, o); break;
    case 1: form_kind<T, R, JW, 1>(D, o); break;
    case 2: form_kind<T, R, JW, 2>(D, o); break;
    default: form_kind<T, R, JW, 3>(D, o); break;
  }
}

template <typename T, int R, int PC, int JW>
__device__ __forceinline__ void consume(T (&acc)[PC][R], const Operands<T>& o, const VGroup& vg,
                                        const Entry<T>* en) {
  T D[JW][R];
  form<T, R, JW>(D, o);
#pragma unroll
  for (int p = 0; p < PC; ++p) {
    const int n = vg.cnt[p];
    for (int e = 0; e < n; ++e) {
      const Entry<T>& E = en[p * ENT_PER + e];
      T k[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) k[q] = E.k[q];
      apply_entry<T, R, JW>(acc[p], D, E.code, k);
    }
  }
}

}  // namespace

template <typename T, int R, int PC, int JW>
__global__ void __launch_bounds__(APPLY_THREADS) k_apply(ApplyArgs<T> A) {
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
  const Entry<T>* en = A.ents + (int64_t)chunk * A.vg_cap * PC * ENT_PER;
  Operands<T> o0, o1;
  if (nv > 0) fetch<T, R, JW>(o0, A, vg[0].g, vg[0].jlo, m0);
  for (int v = 0; v < nv; v += 2) {
    if (v + 1 < nv) fetch<T, R, JW>(o1, A, vg[v + 1].g, vg[v + 1].jlo, m0);
    consume<T, R, PC, JW>(acc, o0, vg[v], en + (int64_t)v * PC * ENT_PER);
    if (v + 1 < nv) {
      if (v + 2 < nv) fetch<T, R, JW>(o0, A, vg[v + 2].g, vg[v + 2].jlo, m0);
      consume<T, R, PC, JW>(acc, o1, vg[v + 1], en + (int64_t)(v + 1) * PC * ENT_PER);
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

hipError_t launch_apply(soap_ctx* c, const Plan& pl, const VGroup* d_vg, const int* d_nvg, const void* d_ent,
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
                       (const Entry<float>*)d_ent, (float*)d_flux};
    hipLaunchKernelGGL((k_apply<float, APPLY_R, PC_F32, APPLY_JW>), grid, dim3(APPLY_THREADS), 0, c->stream, A);
  } else {
    ApplyArgs<double> A{c->P, c->Pstride, c->B, pl.n_ph, pl.n_chunks, c->n_tiles, pl.effect, pl.paired,
                        pl.vg_cap, vec_ok ? 1 : 0,
                        (const double*)c->d_spec[0], (const double*)c->d_spec[1], (const double*)c->d_spec[2],
                        (const double*)c->d_con_spot, (const double*)c->d_con_fac, c->d_Q, d_vg, d_nvg,
                        (const Entry<double>*)d_ent, (double*)d_flux};
    hipLaunchKernelGGL((k_apply<double, APPLY_R, PC_F64, APPLY_JW>), grid, dim3(APPLY_THREADS), 0, c->stream, A);
  }
  return hipGetLastError();
}

}  // namespace soap
