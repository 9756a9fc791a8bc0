// Final spectra of a chunk of phases over a tile of pixels (section 3.3,
// Algorithm 5 with Eqs. 1-4).
//
// With the quiet integrated spectrum Q resident, Eq. 4 gives each phase's
// spectrum as Q minus the summed per-cell differences of the active cells.
// Grouped by disk column and collapsed onto integer pixel offsets (see
// weights.hip), this is
//
//   F[p][m] = Q[m] + sum_g C_g[m] * sum_j K[p][g][j] * S_g[clamp(m - j)]
//
// where group g is either a quiet removal (S_g = quiet spectrum of a mu bin,
// negative taps, C = 1) or an active term (TOT: the region type's spectrum
// with its contrast, FLUX: the quiet spectrum with the contrast, BCONV: the
// region type's spectrum without contrast).  The contrast multiplies after
// the shift, at the output pixel m.
//
// Work split: one block = 256 threads x APPLY_R consecutive pixels (one tile)
// x one chunk of APPLY_PC phases.  The phase accumulators of the chunk live
// in registers; each virtual group's source window and contrast are loaded
// once per tile and reused by every phase of the chunk, so the inner loop is
// only fused multiply-adds.  Taps are walked as runs of <= 4 consecutive
// offsets, dispatched on a wave-uniform code.  The block-to-work mapping
// keeps the chunks of one tile on one XCD so their shared input windows hit
// the same L2.  The final combine adds Q in double.
#include "soap_internal.hpp"

namespace soap {

namespace {

template <int Q0, int W, typename T, int R, int JW>
__device__ __forceinline__ void run_taps(T (&a)[R], const T (&Pq)[JW][R], const T* k) {
  if constexpr (Q0 + W <= JW) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T s = a[r];
#pragma unroll
      for (int q = 0; q < W; ++q) s = fma(k[q], Pq[Q0 + q][r], s);
      a[r] = s;
    }
  }
}

template <typename T, int R, int JW>
__device__ __forceinline__ void apply_entry(T (&a)[R], const T (&Pq)[JW][R], int code, const T* k) {
  static_assert(JW == 8, "dispatch table is written for 8-offset windows");
#define SOAP_CASE(Q0, W) \
  case Q0 * 4 + (W - 1): \
    run_taps<Q0, W, T, R, JW>(a, Pq, k); \
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

template <typename T, int R>
struct VecT;
template <>
struct VecT<float, 4> {
  using type = float4;
};
template <>
struct VecT<double, 4> {
  using type = double4;
};

}  // namespace

template <typename T, int R, int PC, int JW>
__global__ void __launch_bounds__(APPLY_THREADS) k_apply(
    int64_t P, int B, int n_ph, int n_chunks, int n_tiles, int effect, const T* __restrict__ Sq,
    const T* __restrict__ Ss, const T* __restrict__ Sf, const T* __restrict__ Cs, const T* __restrict__ Cf,
    const double* __restrict__ Q, const VGroup* __restrict__ vgs, const int* __restrict__ nvg,
    const Entry<T>* __restrict__ ents, int vg_cap, int ent_cap, T* __restrict__ out) {
  const int total = n_tiles * n_chunks;
  const int per_xcd = (total + 7) / 8;
  const int bid = blockIdx.x;
  const int w = (bid & 7) * per_xcd + (bid >> 3);
  if (w >= total) return;
  const int tile = w / n_chunks;
  const int chunk = w - tile * n_chunks;
  const int64_t m0 = (int64_t)tile * (R * APPLY_THREADS) + (int64_t)threadIdx.x * R;

  T acc[PC][R];
#pragma unroll
  for (int p = 0; p < PC; ++p)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[p][r] = T(0);

  const int nv = nvg[chunk];
  const VGroup* vg = vgs + (int64_t)chunk * vg_cap;
  const Entry<T>* en = ents + (int64_t)chunk * ent_cap;
  for (int v = 0; v < nv; ++v) {
    const int g = vg[v].g;
    const int jlo = vg[v].jlo;
    const int t = g / B;
    const int b = g - t * B;
    const T* src;
    const T* con = nullptr;
    if (t == 0) {
      src = Sq + (int64_t)b * P;
    } else {
      const T* St = (t == SOAP_SPOT ? Ss : Sf) + (int64_t)b * P;
      const T* Ct = nullptr;
      if (Cs) Ct = (t == SOAP_SPOT) ? Cs : Cf + (int64_t)b * P;
      if (effect == SOAP_EFFECT_TOT) {
        src = St;
        con = Ct;
      } else if (effect == SOAP_EFFECT_FLUX) {
        src = Sq + (int64_t)b * P;
        con = Ct;
      } else {
        src = St;
      }
    }
    // Sw[s] = S[clamp(m0 - jlo - (JW - 1) + s)]; offset j = jlo + q reads
    // S[m - j] = Sw[r - q + JW - 1]
    T Sw[R + JW - 1];
    const int64_t base = m0 - jlo - (JW - 1);
#pragma unroll
    for (int s = 0; s < R + JW - 1; ++s) {
      int64_t idx = base + s;
      idx = idx < 0 ? 0 : (idx >= P ? P - 1 : idx);
      Sw[s] = src[idx];
    }
    T Cw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int64_t idx = m0 + r < P ? m0 + r : P - 1;
      Cw[r] = con ? con[idx] : T(1);
    }
    T Pq[JW][R];
#pragma unroll
    for (int q = 0; q < JW; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) Pq[q][r] = Cw[r] * Sw[r - q + JW - 1];

#pragma unroll
    for (int p = 0; p < PC; ++p) {
      const int e0 = vg[v].off[p];
      const int e1 = vg[v].off[p + 1];
      for (int e = e0; e < e1; ++e) {
        const int code = en[e].code;
        T k[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) k[q] = en[e].k[q];
        apply_entry<T, R, JW>(acc[p], Pq, code, k);
      }
    }
  }

  double Qr[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Qr[r] = (m0 + r < P) ? Q[m0 + r] : 0.0;
  const int p0 = chunk * PC;
  const bool full = (m0 + R <= P) && (P % R == 0);
#pragma unroll
  for (int p = 0; p < PC; ++p) {
    if (p0 + p >= n_ph) break;
    T* row = out + (int64_t)(p0 + p) * P;
    T vals[R];
#pragma unroll
    for (int r = 0; r < R; ++r) vals[r] = (T)(Qr[r] + (double)acc[p][r]);
    if (full) {
      using V = typename VecT<T, R>::type;
      V vv;
      vv.x = vals[0];
      vv.y = vals[1];
      vv.z = vals[2];
      vv.w = vals[3];
      *reinterpret_cast<V*>(row + m0) = vv;
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (m0 + r < P) row[m0 + r] = vals[r];
    }
  }
}

hipError_t launch_apply(soap_ctx* c, const VGroup* d_vg, const int* d_nvg, const void* d_ent, int vg_cap,
                        int ent_cap, int n_ph, int effect, void* d_flux) {
  const int n_chunks = (n_ph + APPLY_PC - 1) / APPLY_PC;
  const int n_tiles = (int)((c->P + APPLY_TILE - 1) / APPLY_TILE);
  const int total = n_chunks * n_tiles;
  const int per_xcd = (total + 7) / 8;
  dim3 grid(8 * per_xcd);
  if (c->prec == SOAP_PREC_FP32)
    hipLaunchKernelGGL((k_apply<float, APPLY_R, APPLY_PC, APPLY_JW>), grid, dim3(APPLY_THREADS), 0, c->stream,
                       c->P, c->B, n_ph, n_chunks, n_tiles, effect, (const float*)c->d_spec[0],
                       (const float*)c->d_spec[1], (const float*)c->d_spec[2], (const float*)c->d_con_spot,
                       (const float*)c->d_con_fac, c->d_Q, d_vg, d_nvg, (const Entry<float>*)d_ent, vg_cap,
                       ent_cap, (float*)d_flux);
  else
    hipLaunchKernelGGL((k_apply<double, APPLY_R, APPLY_PC, APPLY_JW>), grid, dim3(APPLY_THREADS), 0,
                       c->stream, c->P, c->B, n_ph, n_chunks, n_tiles, effect, (const double*)c->d_spec[0],
                       (const double*)c->d_spec[1], (const double*)c->d_spec[2], (const double*)c->d_con_spot,
                       (const double*)c->d_con_fac, c->d_Q, d_vg, d_nvg, (const Entry<double>*)d_ent, vg_cap,
                       ent_cap, (double*)d_flux);
  return hipGetLastError();
}

}  // namespace soap
