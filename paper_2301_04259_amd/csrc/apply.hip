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
// The block first copies its chunk's window records (header and dense taps,
// built by the compaction kernel) into LDS, so the main loop reads no
// scalar memory.  For each window of APPLY_JW offsets of one group, every
// thread loads its 11-sample source windows with three 16-byte loads (rows
// are padded with their end samples, so no load needs a bounds check and the
// end-value hold of the interpolation is built in).  Then, offset by offset, the taps
// of each group of four phases that has one there are read from LDS
// (broadcast) and added with fused multiply-adds; a wave-uniform mask test
// skips the other groups.  The next window's loads are issued before the
// current one is consumed.  The block-to-work mapping keeps the chunks of
// one tile on one XCD so their shared input windows hit the same L2, and
// starts the chunks with the most windows first.  The final combine adds Q
// in double.
#include <algorithm>
#include <vector>

#include "soap_internal.hpp"

namespace soap {

namespace {

// 12 consecutive elements from an element-aligned address (the 11-sample
// window of APPLY_R + APPLY_JW - 1 values plus one): three 16-byte loads whose
// type promises only element alignment
typedef float f4e __attribute__((ext_vector_type(4), aligned(4)));
typedef double d2e __attribute__((ext_vector_type(2), aligned(8)));

template <typename T>
struct Win12 {
  T v[12];
};

template <typename T>
__device__ __forceinline__ void load12(Win12<T>& w, const T* p) {
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const f4e f = *reinterpret_cast<const f4e*>(p + 4 * k);
      w.v[4 * k + 0] = f.x;
      w.v[4 * k + 1] = f.y;
      w.v[4 * k + 2] = f.z;
      w.v[4 * k + 3] = f.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const d2e f = *reinterpret_cast<const d2e*>(p + 2 * k);
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
  Win12<T> a, b;  // b is used by paired tables only (D = C A - B)
  T c[4];
};

template <typename T>
struct ApplyArgs {
  int64_t P, Pstride;
  int64_t cs_stride;  // stride of the spot contrast rows per bin (0: one row)
  int B, n_ph, n_chunks, n_tiles, effect, paired, vg_cap, vec_ok, lds_win;
  const T *Sq, *Ss, *Sf, *Cs, *Cf, *ones;
  const double* Q;
  const unsigned char* wins;
  const int* nvg;
  T* out;
};

// header of window v in LDS (type, bin, first offset, group mask)
__device__ __forceinline__ int4 head_raw(const unsigned char* s_win, int v) {
  return *reinterpret_cast<const int4*>(s_win + v * WIN_BYTES);
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Every fetch issues the same loads (a, b for paired tables, c), so that the
// compiler can count outstanding loads exactly and the next window's loads
// stay in flight while the current window is consumed.  Without a contrast
// the c operand comes from a resident row of ones; for the flux effect the
// active operand is the quiet row itself, loaded a second time.
// rows a window reads: active (or quiet) source, quiet source, contrast
template <typename T>
__device__ __forceinline__ void window_rows(const ApplyArgs<T>& A, int4 hr, const T*& src, const T*& sq,
                                            const T*& con, int& jlo) {
  const int t = uni(hr.x), b = uni(hr.y);
  jlo = uni(hr.z);
  const int64_t rs = A.Pstride;  // stride between mu-bin rows
  sq = A.Sq + (int64_t)b * rs;
  con = A.ones;
  if (t == 0) {
    src = sq;
  } else {
    const T* ct = A.ones;
    if (A.Cs) ct = (t == SOAP_SPOT) ? A.Cs + (int64_t)b * A.cs_stride : A.Cf + (int64_t)b * A.Pstride;
    if (A.effect == SOAP_EFFECT_FLUX) {
      src = sq;
      con = ct;
    } else {
      src = (t == SOAP_SPOT ? A.Ss : A.Sf) + (int64_t)b * rs;
      if (A.effect == SOAP_EFFECT_TOT) con = ct;
    }
  }
}

template <typename T, int R, int JW, bool PAIRED>
__device__ __forceinline__ void fetch(Operands<T>& o, const ApplyArgs<T>& A, int4 hr, int64_t m0) {
  const T *src, *sq, *con;
  int jlo;
  window_rows(A, hr, src, sq, con, jlo);
  // window start m0 - jlo - (JW - 1)
  const int64_t at = m0 - jlo - (JW - 1);
  load12(o.a, src + at);
  if (PAIRED) load12(o.b, sq + at);
  load4(o.c, con + m0);
}

// taps of four consecutive phases at one offset, from LDS (all lanes read
// the same address)
template <typename T>
__device__ __forceinline__ void load_taps4(T (&k)[4], const T* p) {
  if constexpr (sizeof(T) == 4) {
    const float4 f = *reinterpret_cast<const float4*>(p);
    k[0] = f.x;
    k[1] = f.y;
    k[2] = f.z;
    k[3] = f.w;
  } else {
    const double2 u = reinterpret_cast<const double2*>(p)[0];
    const double2 w = reinterpret_cast<const double2*>(p)[1];
    k[0] = u.x;
    k[1] = u.y;
    k[2] = w.x;
    k[3] = w.y;
  }
}

// One window: for every offset q with any tap in the chunk, read the taps of
// all phases of that offset from LDS, form the difference row, and let each
// active group of four phases add k * D with fused multiply-adds.
template <typename T, int R, int PC, int JW, bool PAIRED>
__device__ __forceinline__ void consume(T (&acc)[PC][R], const Operands<T>& o, unsigned gm, const T* tw) {
  constexpr int NG = PC / 4;
  constexpr unsigned GMASK = (1u << NG) - 1u;
#pragma unroll
  for (int q = 0; q < JW; ++q) {
    const unsigned nib = (gm >> (q * NG)) & GMASK;
    if (nib == 0u) continue;
    T k[NG][4];
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) load_taps4(k[gi], tw + q * PC + 4 * gi);
    T D[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = r - q + JW - 1;
      D[r] = PAIRED ? fma(o.c[r], o.a.v[s], -o.b.v[s]) : o.c[r] * o.a.v[s];
    }
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      if ((nib >> gi) & 1u) {
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int r = 0; r < R; ++r) acc[4 * gi + p][r] = fma(k[gi][p], D[r], acc[4 * gi + p][r]);
      }
    }
  }
}

}  // namespace

// final combine of one item: Q (double) plus the accumulated differences,
// written with 16-byte stores where the row allows
template <typename T, int R, int PC>
__device__ __forceinline__ void store_item(const ApplyArgs<T>& A, const T (&acc)[PC][R], int chunk, int64_t m0) {
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

// One (tile, chunk) item: the chunk's windows over the tile's pixels, then
// the final combine with Q.  s_win is the block's LDS window staging.
template <typename T, int R, int PC, int JW, bool PAIRED, int THREADS>
__device__ __forceinline__ void apply_item(const ApplyArgs<T>& A, int tile, int chunk, unsigned char* s_win) {
  const int64_t m0 = (int64_t)tile * (R * THREADS) + (int64_t)threadIdx.x * R;

  T acc[PC][R];
#pragma unroll
  for (int p = 0; p < PC; ++p)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[p][r] = T(0);

  const int nv = A.nvg[chunk];
  const unsigned char* gw = A.wins + (int64_t)chunk * A.vg_cap * WIN_BYTES;
  for (int vb = 0; vb < nv; vb += A.lds_win) {
    const int nb = min(A.lds_win, nv - vb);
    if (vb) __syncthreads();  // every wave is done with the previous pass
    {
      const int4* src = reinterpret_cast<const int4*>(gw + (int64_t)vb * WIN_BYTES);
      int4* dst = reinterpret_cast<int4*>(s_win);
      const int n16 = nb * (WIN_BYTES / 16);
      for (int u = threadIdx.x; u < n16; u += THREADS) dst[u] = src[u];
    }
    __syncthreads();
    // Two windows in flight: the loads of the next window are issued before
    // the current one is consumed.  Fetches are unconditional (past the end
    // they repeat the last window and are not consumed), so the compiler
    // can count outstanding loads exactly; headers are read one window
    // ahead of their fetch.
    const int last = nb - 1;
    Operands<T> o0, o1;
    int4 h0 = head_raw(s_win, 0);
    int4 h1 = head_raw(s_win, min(1, last));
    fetch<T, R, JW, PAIRED>(o0, A, h0, m0);
    for (int v = 0; v < nb; v += 2) {
      fetch<T, R, JW, PAIRED>(o1, A, h1, m0);
      const int4 h2 = head_raw(s_win, min(v + 2, last));
      consume<T, R, PC, JW, PAIRED>(acc, o0, (unsigned)uni(h0.w),
                                    reinterpret_cast<const T*>(s_win + v * WIN_BYTES + 16));
      fetch<T, R, JW, PAIRED>(o0, A, h2, m0);
      const int4 h3 = head_raw(s_win, min(v + 3, last));
      if (v + 1 < nb)
        consume<T, R, PC, JW, PAIRED>(acc, o1, (unsigned)uni(h1.w),
                                      reinterpret_cast<const T*>(s_win + (v + 1) * WIN_BYTES + 16));
      h0 = h2;
      h1 = h3;
    }
  }

  store_item<T, R, PC>(A, acc, chunk, m0);
}

// ---- staged variant --------------------------------------------------------
// Each wave stages its own window spans in LDS (the wave's 256 pixels + 12
// source samples, the quiet samples, 256 contrast values) with coalesced
// 16-byte loads, double-buffered: the next window's spans are loaded into
// registers while the current window is consumed from LDS, then written to
// the other buffer.  Lanes read their 12-sample windows from LDS instead of
// loading overlapping windows from memory.  The spans are private to the
// wave, so no block barrier is needed per window.  Tile of APPLY_TILE pixels
// (256 threads, 4 waves).
constexpr int WV_PIX = 64 * APPLY_R;   // pixels of one wave
constexpr int WV_SPAN = WV_PIX + 16;   // + 12 samples, 16-byte rows
constexpr int WV_BUF = 2 * WV_SPAN + WV_PIX;

template <typename T>
__device__ __forceinline__ void load4e(T* x, const T* p) {
  if constexpr (sizeof(T) == 4) {
    const f4e f = *reinterpret_cast<const f4e*>(p);
    x[0] = f.x;
    x[1] = f.y;
    x[2] = f.z;
    x[3] = f.w;
  } else {
    const d2e u = *reinterpret_cast<const d2e*>(p);
    const d2e w = *reinterpret_cast<const d2e*>(p + 2);
    x[0] = u.x;
    x[1] = u.y;
    x[2] = w.x;
    x[3] = w.y;
  }
}

// 4 consecutive elements to / from 16-byte-aligned LDS
template <typename T>
__device__ __forceinline__ void lds_put4(T* p, const T* x) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(x[0], x[1], x[2], x[3]);
  } else {
    reinterpret_cast<double2*>(p)[0] = make_double2(x[0], x[1]);
    reinterpret_cast<double2*>(p)[1] = make_double2(x[2], x[3]);
  }
}

template <typename T>
__device__ __forceinline__ void lds_get4(T* x, const T* p) {
  if constexpr (sizeof(T) == 4) {
    const float4 f = *reinterpret_cast<const float4*>(p);
    x[0] = f.x;
    x[1] = f.y;
    x[2] = f.z;
    x[3] = f.w;
  } else {
    const double2 u = reinterpret_cast<const double2*>(p)[0];
    const double2 w = reinterpret_cast<const double2*>(p)[1];
    x[0] = u.x;
    x[1] = u.y;
    x[2] = w.x;
    x[3] = w.y;
  }
}

// one lane's share of its wave's spans: a[0..3] (and a[4..7], the 12
// samples past the wave's pixels, for lanes 0..2), the same for the quiet
// row b, and 4 contrast values
template <typename T>
struct Stage {
  T a[8], b[8], c[4];
};

template <typename T, int JW, bool PAIRED>
__device__ __forceinline__ void stage_load(Stage<T>& g, const ApplyArgs<T>& A, int4 hr, int64_t mw, int lane) {
  const T *src, *sq, *con;
  int jlo;
  window_rows(A, hr, src, sq, con, jlo);
  const int64_t at = mw - jlo - (JW - 1);
  const int i = 4 * lane;
  load4e(&g.a[0], src + at + i);
  if (PAIRED) load4e(&g.b[0], sq + at + i);
  if (lane < 3) {
    load4e(&g.a[4], src + at + WV_PIX + i);
    if (PAIRED) load4e(&g.b[4], sq + at + WV_PIX + i);
  }
  load4e(&g.c[0], con + mw + i);
}

template <typename T, bool PAIRED>
__device__ __forceinline__ void stage_store(T* buf, const Stage<T>& g, int lane) {
  const int i = 4 * lane;
  lds_put4(buf + i, &g.a[0]);
  if (PAIRED) lds_put4(buf + WV_SPAN + i, &g.b[0]);
  if (lane < 3) {
    lds_put4(buf + WV_PIX + i, &g.a[4]);
    if (PAIRED) lds_put4(buf + WV_SPAN + WV_PIX + i, &g.b[4]);
  }
  lds_put4(buf + 2 * WV_SPAN + i, &g.c[0]);
}

template <typename T, bool PAIRED>
__device__ __forceinline__ void stage_read(Operands<T>& o, const T* buf, int lane) {
  const int i = 4 * lane;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lds_get4(&o.a.v[4 * k], buf + i + 4 * k);
    if (PAIRED) lds_get4(&o.b.v[4 * k], buf + WV_SPAN + i + 4 * k);
  }
  lds_get4(&o.c[0], buf + 2 * WV_SPAN + i);
}

// the wave's own LDS writes are visible to its later reads
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int R, int PC, int JW, bool PAIRED>
__device__ __forceinline__ void apply_item_staged(const ApplyArgs<T>& A, int tile, int chunk, unsigned char* s_win) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t mw = (int64_t)tile * APPLY_TILE + (int64_t)wave * WV_PIX;
  const int64_t m0 = mw + (int64_t)lane * R;
  T* stg = reinterpret_cast<T*>(s_win + (size_t)A.lds_win * WIN_BYTES) + (size_t)wave * 2 * WV_BUF;

  T acc[PC][R];
#pragma unroll
  for (int p = 0; p < PC; ++p)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[p][r] = T(0);

  const int nv = A.nvg[chunk];
  const unsigned char* gw = A.wins + (int64_t)chunk * A.vg_cap * WIN_BYTES;
  for (int vb = 0; vb < nv; vb += A.lds_win) {
    const int nb = min(A.lds_win, nv - vb);
    if (vb) __syncthreads();  // every wave is done with the previous pass
    {
      const int4* src = reinterpret_cast<const int4*>(gw + (int64_t)vb * WIN_BYTES);
      int4* dst = reinterpret_cast<int4*>(s_win);
      const int n16 = nb * (WIN_BYTES / 16);
      for (int u = threadIdx.x; u < n16; u += APPLY_THREADS) dst[u] = src[u];
    }
    __syncthreads();
    Stage<T> g;
    stage_load<T, JW, PAIRED>(g, A, head_raw(s_win, 0), mw, lane);
    stage_store<T, PAIRED>(stg, g, lane);
    wave_sync();
    for (int v = 0; v < nb; ++v) {
      const bool more = v + 1 < nb;  // uniform
      if (more) stage_load<T, JW, PAIRED>(g, A, head_raw(s_win, v + 1), mw, lane);
      Operands<T> o;
      stage_read<T, PAIRED>(o, stg + (v & 1) * WV_BUF, lane);
      consume<T, R, PC, JW, PAIRED>(acc, o, (unsigned)uni(head_raw(s_win, v).w),
                                    reinterpret_cast<const T*>(s_win + v * WIN_BYTES + 16));
      if (more) stage_store<T, PAIRED>(stg + ((v + 1) & 1) * WV_BUF, g, lane);
      wave_sync();
    }
  }
  store_item<T, R, PC>(A, acc, chunk, m0);
}

// Blocks are dealt to the 8 XCDs in turn (block index mod 8).  Each XCD
// owns a contiguous range of tiles, so the chunks of a tile share its L2,
// and walks its (chunk, tile) items heaviest chunk first (most windows), so
// that the long blocks start early and the short ones fill the end.  seq8 is
// the block's index within the configuration's 8 * ceil(n_tiles / 8) *
// n_chunks slots; returns false for a slot with no item.
template <typename T>
__device__ __forceinline__ bool map_item(const ApplyArgs<T>& A, int seq8, int* s_order, int* tile, int* chunk) {
  const int xcd = seq8 & 7;
  const int seq = seq8 >> 3;
  const int tpx = (A.n_tiles + 7) / 8;
  const int t0 = xcd * tpx;
  const int nt = min(A.n_tiles, t0 + tpx) - t0;
  if (nt <= 0 || seq >= nt * A.n_chunks) return false;
  const int rank = seq / nt;
  *tile = t0 + (seq - rank * nt);
  *chunk = rank;
  if (A.n_chunks <= APPLY_RANKED) {
    // rank of each chunk by window count (ties in chunk order)
    const int c = threadIdx.x;
    const int wc = c < A.n_chunks ? A.nvg[c] : 0;
    if (c < A.n_chunks) s_order[c] = wc;  // window counts, then the order
    __syncthreads();
    int r = 0;
    if (c < A.n_chunks)
      for (int d = 0; d < A.n_chunks; ++d) {
        const int wd = s_order[d];
        r += (wd > wc || (wd == wc && d < c)) ? 1 : 0;
      }
    __syncthreads();
    if (c < A.n_chunks) s_order[r] = c;
    __syncthreads();
    *chunk = s_order[rank];
  }
  return true;
}

template <typename T, int R, int PC, int JW, bool PAIRED, int THREADS, bool STAGED>
__global__ void __launch_bounds__(THREADS, sizeof(T) == 4 ? 3 : 2) k_apply(ApplyArgs<T> A) {
  static_assert(R == 4 && JW == 8, "window loads are written for 4 pixels x 8 offsets");
  static_assert(PC % 4 == 0 && JW * PC * sizeof(T) == WIN_TAP_BYTES, "record layout");
  extern __shared__ __align__(16) unsigned char s_win[];  // [lds_win][WIN_BYTES]
  __shared__ int s_order[APPLY_RANKED];
  int tile, chunk;
  if (!map_item(A, blockIdx.x, s_order, &tile, &chunk)) return;
  if constexpr (STAGED)
    apply_item_staged<T, R, PC, JW, PAIRED>(A, tile, chunk, s_win);
  else
    apply_item<T, R, PC, JW, PAIRED, THREADS>(A, tile, chunk, s_win);
}

// Batched form: one launch over the items of many configurations (each with
// its own arguments).  Configuration i owns the slots item_off[i] ..
// item_off[i+1] - 1, a multiple of 8 starting at a multiple of 8, mapped as
// in k_apply.
template <typename T, int R, int PC, int JW, bool PAIRED, int THREADS>
__global__ void __launch_bounds__(THREADS, sizeof(T) == 4 ? 3 : 2)
    k_apply_batch(const ApplyArgs<T>* __restrict__ args, const int* __restrict__ item_off, int n_cfg) {
  extern __shared__ __align__(16) unsigned char s_win[];
  __shared__ int s_order[APPLY_RANKED];
  const int b = blockIdx.x;
  int lo = 0, hi = n_cfg;  // last cfg with item_off[cfg] <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (item_off[mid] <= b) lo = mid;
    else hi = mid;
  }
  const ApplyArgs<T> A = args[lo];
  int tile, chunk;
  if (!map_item(A, b - item_off[lo], s_order, &tile, &chunk)) return;
  apply_item<T, R, PC, JW, PAIRED, THREADS>(A, tile, chunk, s_win);
}

namespace {

template <typename T, bool PAIRED, int PC>
hipError_t launch_apply_t(soap_ctx* c, const Plan& pl, const ApplyArgs<T>& A0, int threads, bool staged,
                          hipStream_t st) {
  ApplyArgs<T> A = A0;
  if (staged) threads = APPLY_THREADS;
  const int tile = APPLY_R * threads;
  A.n_tiles = (int)((c->P + tile - 1) / tile);
  const int tpx = (A.n_tiles + 7) / 8;
  const dim3 grid(8 * tpx * pl.n_chunks);
  if (staged) {
    // the staging buffers take their share of at most 60 KB per block
    const size_t stg = (size_t)(APPLY_THREADS / 64) * 2 * WV_BUF * sizeof(T);
    A.lds_win = std::max(1, std::min<int>(A.lds_win, (int)((60 * 1024 - stg) / WIN_BYTES)));
    const size_t lds = (size_t)A.lds_win * WIN_BYTES + stg;
    hipLaunchKernelGGL((k_apply<T, APPLY_R, PC, APPLY_JW, PAIRED, 256, true>), grid, dim3(256), lds, st, A);
    return hipGetLastError();
  }
  const size_t lds = (size_t)A.lds_win * WIN_BYTES;
  switch (threads) {
    case 64:
      hipLaunchKernelGGL((k_apply<T, APPLY_R, PC, APPLY_JW, PAIRED, 64, false>), grid, dim3(64), lds, st, A);
      break;
    case 128:
      hipLaunchKernelGGL((k_apply<T, APPLY_R, PC, APPLY_JW, PAIRED, 128, false>), grid, dim3(128), lds, st, A);
      break;
    case 512:
      hipLaunchKernelGGL((k_apply<T, APPLY_R, PC, APPLY_JW, PAIRED, 512, false>), grid, dim3(512), lds, st, A);
      break;
    default:
      hipLaunchKernelGGL((k_apply<T, APPLY_R, PC, APPLY_JW, PAIRED, 256, false>), grid, dim3(256), lds, st, A);
      break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_apply(soap_ctx* c, const Plan& pl, const void* d_win, const int* d_nvg, void* d_flux) {
  return launch_apply_shape(c, pl, d_win, d_nvg, d_flux, c->tune_threads, c->tune_lds_win, c->tune_staged != 0,
                            c->stream);
}

hipError_t launch_apply_shape(soap_ctx* c, const Plan& pl, const void* d_win, const int* d_nvg, void* d_flux,
                              int threads, int lds_win, bool staged, hipStream_t st) {
  const bool vec_ok = (c->P % APPLY_R == 0) &&
                      (reinterpret_cast<uintptr_t>(d_flux) % (APPLY_R * c->esize) == 0);
  lds_win = std::max(1, std::min(pl.vg_cap, lds_win));
  const unsigned char* w = static_cast<const unsigned char*>(d_win);
  if (c->prec == SOAP_PREC_FP32) {
    ApplyArgs<float> A{c->P, c->Pstride, c->con_spot_stride, c->B, pl.n_ph, pl.n_chunks, 0, pl.effect, pl.paired, pl.vg_cap,
                       vec_ok ? 1 : 0, lds_win,
                       (const float*)c->d_spec[0], (const float*)c->d_spec[1], (const float*)c->d_spec[2],
                       (const float*)c->d_con_spot, (const float*)c->d_con_fac, (const float*)c->d_ones, c->d_Q, w, d_nvg,
                       (float*)d_flux};
    return pl.paired ? launch_apply_t<float, true, PC_F32>(c, pl, A, threads, staged, st)
                     : launch_apply_t<float, false, PC_F32>(c, pl, A, threads, staged, st);
  }
  ApplyArgs<double> A{c->P, c->Pstride, c->con_spot_stride, c->B, pl.n_ph, pl.n_chunks, 0, pl.effect, pl.paired,
                      pl.vg_cap, vec_ok ? 1 : 0, lds_win,
                      (const double*)c->d_spec[0], (const double*)c->d_spec[1], (const double*)c->d_spec[2],
                      (const double*)c->d_con_spot, (const double*)c->d_con_fac, (const double*)c->d_ones, c->d_Q, w, d_nvg,
                      (double*)d_flux};
  return pl.paired ? launch_apply_t<double, true, PC_F64>(c, pl, A, threads, staged, st)
                   : launch_apply_t<double, false, PC_F64>(c, pl, A, threads, staged, st);
}

// ---- batched shift-and-sum over many configurations ------------------------

namespace {

template <typename T>
ApplyArgs<T> make_args(const ApplyBatchCfg& q) {
  soap_ctx* c = q.c;
  const bool vec_ok =
      (c->P % APPLY_R == 0) && (reinterpret_cast<uintptr_t>(q.flux) % (APPLY_R * c->esize) == 0);
  ApplyArgs<T> A{c->P, c->Pstride, c->con_spot_stride, c->B, q.pl.n_ph, q.pl.n_chunks, (int)((c->P + APPLY_TILE - 1) / APPLY_TILE),
                 q.pl.effect, q.pl.paired, q.pl.vg_cap, vec_ok ? 1 : 0,
                 std::max(1, std::min(q.pl.vg_cap, APPLY_LDS_WIN)),
                 (const T*)c->d_spec[0], (const T*)c->d_spec[1], (const T*)c->d_spec[2], (const T*)c->d_con_spot,
                 (const T*)c->d_con_fac, (const T*)c->d_ones, c->d_Q, static_cast<const unsigned char*>(q.win), q.nvg,
                 (T*)q.flux};
  return A;
}

template <typename T>
hipError_t upload_t(const ApplyBatchCfg* cfgs, int n, void* d_buf, ApplyBatchGroup* g) {
  std::vector<ApplyArgs<T>> args(n);
  std::vector<int> off(n + 1, 0);
  int lw = 1;
  for (int i = 0; i < n; ++i) {
    args[i] = make_args<T>(cfgs[i]);
    off[i + 1] = off[i] + 8 * ((args[i].n_tiles + 7) / 8) * args[i].n_chunks;  // whole XCD rounds
    lw = std::max(lw, args[i].lds_win);
  }
  g->n_cfg = n;
  g->n_items = off[n];
  g->lds_win = lw;
  g->args = d_buf;
  g->off = static_cast<unsigned char*>(d_buf) + 256 * ((sizeof(ApplyArgs<T>) * n + 255) / 256);
  hipError_t e = hipMemcpy(g->args, args.data(), sizeof(ApplyArgs<T>) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemcpy(g->off, off.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice);
}

}  // namespace

size_t apply_batch_bytes(int n) {
  return 256 * ((sizeof(ApplyArgs<double>) * n + 255) / 256) + sizeof(int) * (n + 1) + 256;
}

hipError_t apply_batch_upload(const ApplyBatchCfg* cfgs, int n, void* d_buf, ApplyBatchGroup* g) {
  g->fp32 = cfgs[0].c->prec == SOAP_PREC_FP32;
  g->paired = cfgs[0].pl.paired != 0;
  return g->fp32 ? upload_t<float>(cfgs, n, d_buf, g) : upload_t<double>(cfgs, n, d_buf, g);
}

hipError_t apply_batch_launch(const ApplyBatchGroup& g, hipStream_t st) {
  if (g.n_items <= 0) return hipSuccess;
  const dim3 grid((unsigned)g.n_items), block(APPLY_THREADS);
  const size_t lds = (size_t)g.lds_win * WIN_BYTES;
  const int* off = static_cast<const int*>(g.off);
  if (g.fp32) {
    const auto* a = static_cast<const ApplyArgs<float>*>(g.args);
    if (g.paired)
      hipLaunchKernelGGL((k_apply_batch<float, APPLY_R, PC_F32, APPLY_JW, true, APPLY_THREADS>), grid, block, lds,
                         st, a, off, g.n_cfg);
    else
      hipLaunchKernelGGL((k_apply_batch<float, APPLY_R, PC_F32, APPLY_JW, false, APPLY_THREADS>), grid, block, lds,
                         st, a, off, g.n_cfg);
  } else {
    const auto* a = static_cast<const ApplyArgs<double>*>(g.args);
    if (g.paired)
      hipLaunchKernelGGL((k_apply_batch<double, APPLY_R, PC_F64, APPLY_JW, true, APPLY_THREADS>), grid, block, lds,
                         st, a, off, g.n_cfg);
    else
      hipLaunchKernelGGL((k_apply_batch<double, APPLY_R, PC_F64, APPLY_JW, false, APPLY_THREADS>), grid, block,
                         lds, st, a, off, g.n_cfg);
  }
  return hipGetLastError();
}

}  // namespace soap
