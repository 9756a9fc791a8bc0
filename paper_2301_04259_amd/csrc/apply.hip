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
// Work split: one block of APPLY_WAVES waves per (tile of APPLY_WAVES x 64
// x R pixels, chunk of PC phases); each wave owns 64 x R consecutive pixels
// of the tile (R per lane) and walks every window of the chunk's list over
// them, with R x PC accumulators per lane in registers.  The block copies
// the chunk's window records (header and dense taps of APPLY_JW offsets,
// built by the compaction kernel) into LDS, APPLY_LDS_WIN records per pass
// with a barrier between passes, so the taps reach every lane as broadcast
// LDS reads.  For each window a lane loads the R + APPLY_JW - 1 source
// samples its pixels need (and as many quiet samples for paired tables) and
// its R contrast values (rows are padded with their end samples, so no load
// needs a bounds check and the end-value hold of the interpolation is built
// in); then, offset by offset, each pair of phases with a tap there adds
// k * D with fused multiply-adds, and a wave-uniform mask test skips the
// other pairs.  The loads of the next DEP - 1 windows are in flight while a
// window is consumed.  The block-to-work mapping keeps the chunks of one
// tile on one XCD so their shared input windows hit the same L2, and either
// starts the chunks with the most windows first or walks the tiles in
// order.  The final store adds Q in double.  Every pixel's sum runs over the
// windows in list order, so results repeat bit for bit whatever the
// pipeline depth or item order.
#include <algorithm>
#include <vector>

#include "soap_internal.hpp"

namespace soap {

namespace {

// The R + APPLY_JW - 1 consecutive elements of a window from an
// element-aligned address: 16-byte loads and one shorter load for the rest,
// whose types promise only element alignment.  Every loaded element is used:
// a loaded register that the program never reads may be reused by the
// compiler while its load is still in flight, which makes the wave wait for
// that load.
typedef float f4e __attribute__((ext_vector_type(4), aligned(4)));
typedef float f3e __attribute__((ext_vector_type(3), aligned(4)));
typedef double d2e __attribute__((ext_vector_type(2), aligned(8)));

template <typename T, int PC>
constexpr int win_n() {
  return ApplyShape<T, PC>::R + APPLY_JW - 1;
}

template <typename T, int PC>
__device__ __forceinline__ void load_win(T (&w)[(win_n<T, PC>())], const T* p) {
  constexpr int N = win_n<T, PC>();
  if constexpr (sizeof(T) == 4) {
    static_assert(N % 4 == 3, "16-byte loads and one 12-byte load");
#pragma unroll
    for (int k = 0; k + 4 <= N; k += 4) {
      const f4e f = *reinterpret_cast<const f4e*>(p + k);
      w[k] = f.x;
      w[k + 1] = f.y;
      w[k + 2] = f.z;
      w[k + 3] = f.w;
    }
    const f3e g = *reinterpret_cast<const f3e*>(p + N - 3);
    w[N - 3] = g.x;
    w[N - 2] = g.y;
    w[N - 1] = g.z;
  } else {
    static_assert(N % 2 == 1, "16-byte loads and one 8-byte load");
#pragma unroll
    for (int k = 0; k + 2 <= N; k += 2) {
      const d2e f = *reinterpret_cast<const d2e*>(p + k);
      w[k] = f.x;
      w[k + 1] = f.y;
    }
    w[N - 1] = p[N - 1];
  }
}

// R consecutive elements from 16-byte-aligned memory
template <typename T, int PC>
__device__ __forceinline__ void load_px(T (&c)[(ApplyShape<T, PC>::R)], const T* p) {
  constexpr int R = ApplyShape<T, PC>::R;
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < R; k += 4) {
      const float4 f = *reinterpret_cast<const float4*>(p + k);
      c[k] = f.x;
      c[k + 1] = f.y;
      c[k + 2] = f.z;
      c[k + 3] = f.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < R; k += 2) {
      const double2 f = *reinterpret_cast<const double2*>(p + k);
      c[k] = f.x;
      c[k + 1] = f.y;
    }
  }
}

// operands of one window: D[q][r] = Ca[r] * A[m_r - j] - B[m_r - j],
// j = jlo + q, with window sample s = r - q + APPLY_JW - 1
template <typename T, int PC>
struct Operands {
  T a[(win_n<T, PC>())], b[(win_n<T, PC>())];  // b is used by paired tables only (D = C A - B)
  T c[(ApplyShape<T, PC>::R)];
};

template <typename T>
struct ApplyArgs {
  int64_t P, Pstride;
  int64_t cs_stride;  // stride of the spot contrast rows per bin (0: one row)
  int B, n_ph, n_chunks, n_tiles, effect, paired, vg_cap, vec_ok, order;
  const T *Sq, *Ss, *Sf, *Cs, *Cf, *ones;
  const double* Q;
  const unsigned char* wins;
  const int* nvg;
  T* out;
};

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Rows a window reads: active (or quiet) source, quiet source, contrast.
// Every fetch issues the same loads (a, b for paired tables, c), so that the
// compiler can count outstanding loads exactly and the next windows' loads
// stay in flight while the current window is consumed.  Without a contrast
// the c operand comes from a resident row of ones; for the flux effect the
// active operand is the quiet row itself, loaded a second time.  EFF is the
// effect when known at compile time (-1: read from the arguments).  Row
// offsets fit 32 bits (mu bins x padded row length), so the selection is a
// few scalar multiplies and selects.
template <typename T, int EFF>
__device__ __forceinline__ void window_rows(const ApplyArgs<T>& A, int4 hr, const T*& src, const T*& sq,
                                            const T*& con, int& jlo) {
  const int t = uni(hr.x), b = uni(hr.y);
  jlo = uni(hr.z);
  const int eff = EFF >= 0 ? EFF : A.effect;
  const int off = b * (int)A.Pstride;  // row b of a [B][Pstride] table
  sq = A.Sq + off;
  const T* st = (t == SOAP_SPOT ? A.Ss : A.Sf) + off;
  const T* ct = A.ones;
  if (A.Cs) ct = t == SOAP_SPOT ? A.Cs + (A.cs_stride ? off : 0) : A.Cf + off;
  const bool quiet = t == 0;
  src = (quiet || eff == SOAP_EFFECT_FLUX) ? sq : st;
  con = (quiet || eff == SOAP_EFFECT_BCONV) ? A.ones : ct;
}

// mt: first pixel of the tile (uniform); lo: the lane's first pixel within
// it.  The uniform part of every address is formed in SGPRs, so each load
// takes a scalar base and a 32-bit per-lane offset.
template <typename T, int PC, int EFF, bool PAIRED>
__device__ __forceinline__ void fetch(Operands<T, PC>& o, const ApplyArgs<T>& A, int4 hr, int64_t mt, unsigned lo) {
  const T *src, *sq, *con;
  int jlo;
  window_rows<T, EFF>(A, hr, src, sq, con, jlo);
  // window start m - jlo - (JW - 1)
  const int64_t at = mt - jlo - (APPLY_JW - 1);
  load_win<T, PC>(o.a, (src + at) + lo);
  if (PAIRED) load_win<T, PC>(o.b, (sq + at) + lo);
  load_px<T, PC>(o.c, (con + mt) + lo);
}

// One window: for every offset q with a tap in the chunk, read the taps of
// all phases at that offset from LDS (every lane reads the same address),
// form the difference row, and let each pair of phases with a tap there add
// k * D with fused multiply-adds.
template <typename T, int PC, bool PAIRED>
__device__ __forceinline__ void consume(T (&acc)[PC][(ApplyShape<T, PC>::R)], const Operands<T, PC>& o, unsigned gm,
                                        const T* tw) {
  constexpr int R = ApplyShape<T, PC>::R, JW = APPLY_JW, NP = PC / 2;
  constexpr unsigned PMASK = (1u << NP) - 1u;
#pragma unroll
  for (int q = 0; q < JW; ++q) {
    const unsigned bits = (gm >> (q * NP)) & PMASK;
    if (bits == 0u) continue;
    T k[PC];
#pragma unroll
    for (int p = 0; p < PC; ++p) k[p] = tw[q * PC + p];
    T D[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = r - q + JW - 1;
      D[r] = PAIRED ? fma(o.c[r], o.a[s], -o.b[s]) : o.c[r] * o.a[s];
    }
#pragma unroll
    for (int pi = 0; pi < NP; ++pi) {
      if (__builtin_expect((bits >> pi) & 1u, 1)) {
#pragma unroll
        for (int p = 2 * pi; p < 2 * pi + 2; ++p)
#pragma unroll
          for (int r = 0; r < R; ++r) acc[p][r] = fma(k[p], D[r], acc[p][r]);
      }
    }
  }
}

}  // namespace

// final combine of one item: Q (double) plus the accumulated differences,
// written with 16-byte stores where the row allows
template <typename T, int PC>
__device__ __forceinline__ void store_item(const ApplyArgs<T>& A, const T (&acc)[PC][(ApplyShape<T, PC>::R)], int chunk,
                                           int64_t m0) {
  constexpr int R = ApplyShape<T, PC>::R;
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
#pragma unroll
        for (int r = 0; r < R; r += 4)
          *reinterpret_cast<float4*>(row + m0 + r) = make_float4(vals[r], vals[r + 1], vals[r + 2], vals[r + 3]);
      } else {
#pragma unroll
        for (int r = 0; r < R; r += 2) *reinterpret_cast<double2*>(row + m0 + r) = make_double2(vals[r], vals[r + 1]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (m0 + r < A.P) row[m0 + r] = vals[r];
    }
  }
}

// One (tile, chunk) item: each wave walks all of the chunk's windows over its
// own 64 x APPLY_R pixels of the tile (DEP windows in flight: the loads of
// window v + DEP - 1 are issued before window v is consumed; fetches are
// unconditional, past the end they repeat the last window and are not
// consumed, so the compiler can count outstanding loads exactly; each header
// is read one step ahead of its fetch).  The block stages the records
// APPLY_LDS_WIN at a time.  Then Q is added and the spectra stored.
template <typename T, int PC, bool PAIRED, int EFF, int DEP>
__device__ __forceinline__ void apply_item(const ApplyArgs<T>& A, int tile, int chunk, unsigned char* lds) {
  constexpr int R = ApplyShape<T, PC>::R, WB = ApplyShape<T, PC>::WB;
  const int64_t mt = (int64_t)tile * ApplyShape<T, PC>::TILE;
  const unsigned lo = threadIdx.x * R;

  T acc[PC][R];
#pragma unroll
  for (int p = 0; p < PC; ++p)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[p][r] = T(0);

  const int nv = A.nvg[chunk];
  const unsigned char* gw = A.wins + (int64_t)chunk * A.vg_cap * WB;
  for (int vb = 0; vb < nv; vb += APPLY_LDS_WIN) {
    const int nb = min(APPLY_LDS_WIN, nv - vb);
    if (vb) __syncthreads();  // every wave is done with the previous pass
    {
      const int4* src = reinterpret_cast<const int4*>(gw + (int64_t)vb * WB);
      int4* dst = reinterpret_cast<int4*>(lds);
      const int n16 = nb * (WB / 16);
      for (int u = threadIdx.x; u < n16; u += APPLY_WAVES * 64) dst[u] = src[u];
    }
    __syncthreads();
    const int last = nb - 1;
    auto head = [&](int v) { return *reinterpret_cast<const int4*>(lds + min(v, last) * WB); };
    Operands<T, PC> o[DEP];
    int4 h[DEP];
#pragma unroll
    for (int i = 0; i < DEP; ++i) h[i] = head(i);
#pragma unroll
    for (int i = 0; i + 1 < DEP; ++i) fetch<T, PC, EFF, PAIRED>(o[i], A, h[i], mt, lo);
    for (int v0 = 0; v0 < nb; v0 += DEP) {
#pragma unroll
      for (int d = 0; d < DEP; ++d) {
        const int nxt = (d + DEP - 1) % DEP;  // slot of window v0 + d + DEP - 1
        fetch<T, PC, EFF, PAIRED>(o[nxt], A, h[nxt], mt, lo);
        const int4 hc = h[d];
        h[d] = head(v0 + d + DEP);
        if (v0 + d < nb)
          consume<T, PC, PAIRED>(acc, o[d], (unsigned)uni(hc.w), reinterpret_cast<const T*>(lds + (v0 + d) * WB + 16));
      }
    }
  }
  store_item<T, PC>(A, acc, chunk, mt + lo);
}

// Blocks are dealt to the 8 XCDs in turn (block index mod 8).  Each XCD
// owns a contiguous range of tiles, so the chunks of a tile share its L2,
// and walks its (chunk, tile) items either heaviest chunk first (most
// windows: the long blocks start early and the short ones fill the end) or
// tile by tile (the chunks of a tile run together).  seq8 is
// the block's index within the configuration's 8 * ceil(n_tiles / 8) *
// n_chunks slots; returns false for a slot with no item.
template <typename T>
__device__ __forceinline__ bool map_item(const ApplyArgs<T>& A, int seq8, int* tile, int* chunk) {
  const int xcd = seq8 & 7;
  const int seq = seq8 >> 3;
  const int tpx = (A.n_tiles + 7) / 8;
  const int t0 = xcd * tpx;
  const int nt = min(A.n_tiles, t0 + tpx) - t0;
  if (nt <= 0 || seq >= nt * A.n_chunks) return false;
  if (A.order == 1) {  // tile by tile
    *tile = t0 + seq / A.n_chunks;
    *chunk = seq % A.n_chunks;
    return true;
  }
  const int rank = seq / nt;
  *tile = t0 + (seq - rank * nt);
  *chunk = rank;
  if (A.n_chunks <= APPLY_RANKED) {
    // each wave ranks the chunks by window count (ties in chunk order): one
    // chunk per lane, the counts exchanged across lanes, and takes the chunk
    // of the wanted rank
    const int c = threadIdx.x & 63;
    const int wc = c < A.n_chunks ? A.nvg[c] : 0;
    int r = 0;
    for (int d = 0; d < A.n_chunks; ++d) {
      const int wd = __builtin_amdgcn_readlane(wc, d);
      r += (wd > wc || (wd == wc && d < c)) ? 1 : 0;
    }
    const unsigned long long hit = __ballot(c < A.n_chunks && r == rank);
    *chunk = uni(__ffsll((long long)hit) - 1);
  }
  return true;
}

// waves per SIMD the register budget is sized for: three with two windows
// in flight (FP32, or FP64 with its 2-pixel lanes), two where more registers
// are needed (FP64 with 4-pixel lanes, a third window in flight, the effect
// read at run time)
template <typename T, int PC, int EFF, int DEP>
constexpr int apply_occupancy() {
  return ((sizeof(T) == 4 || PC == PC_F64_WIDE) && DEP == 2 && EFF >= 0) ? 3 : 2;
}

template <typename T, int PC, bool PAIRED, int EFF, int DEP>
__global__ void __launch_bounds__(APPLY_WAVES * 64, (apply_occupancy<T, PC, EFF, DEP>())) k_apply(ApplyArgs<T> A) {
  __shared__ __align__(16) unsigned char lds[APPLY_LDS_WIN * ApplyShape<T, PC>::WB];
  int tile, chunk;
  if (!map_item(A, blockIdx.x, &tile, &chunk)) return;
  apply_item<T, PC, PAIRED, EFF, DEP>(A, tile, chunk, lds);
}

// Batched form: one launch over the items of many configurations (each with
// its own arguments, all with PC phases per chunk).  Configuration i owns the
// slots item_off[i] .. item_off[i+1] - 1, a multiple of 8 starting at a
// multiple of 8, mapped as in k_apply.
template <typename T, int PC, bool PAIRED, int EFF, int DEP>
__global__ void __launch_bounds__(APPLY_WAVES * 64, (apply_occupancy<T, PC, EFF, DEP>()))
    k_apply_batch(const ApplyArgs<T>* __restrict__ args, const int* __restrict__ item_off, int n_cfg) {
  __shared__ __align__(16) unsigned char lds[APPLY_LDS_WIN * ApplyShape<T, PC>::WB];
  const int b = blockIdx.x;
  int lo = 0, hi = n_cfg;  // last cfg with item_off[cfg] <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (item_off[mid] <= b) lo = mid;
    else hi = mid;
  }
  const ApplyArgs<T> A = args[lo];
  int tile, chunk;
  if (!map_item(A, b - item_off[lo], &tile, &chunk)) return;
  apply_item<T, PC, PAIRED, EFF, DEP>(A, tile, chunk, lds);
}

namespace {

template <typename T, int PC, bool PAIRED, int EFF>
hipError_t launch_eff(const ApplyArgs<T>& A, int depth, dim3 grid, hipStream_t st) {
  const dim3 block(APPLY_WAVES * 64);
  if (depth >= 3)
    hipLaunchKernelGGL((k_apply<T, PC, PAIRED, EFF, 3>), grid, block, 0, st, A);
  else
    hipLaunchKernelGGL((k_apply<T, PC, PAIRED, EFF, 2>), grid, block, 0, st, A);
  return hipGetLastError();
}

template <typename T, int PC, bool PAIRED>
hipError_t launch_apply_t(const Plan& pl, const ApplyArgs<T>& A, int depth, hipStream_t st) {
  const int tpx = (A.n_tiles + 7) / 8;
  const dim3 grid(8 * tpx * pl.n_chunks);
  switch (pl.effect) {
    case SOAP_EFFECT_FLUX:
      return launch_eff<T, PC, PAIRED, SOAP_EFFECT_FLUX>(A, depth, grid, st);
    case SOAP_EFFECT_BCONV:
      return launch_eff<T, PC, PAIRED, SOAP_EFFECT_BCONV>(A, depth, grid, st);
    default:
      return launch_eff<T, PC, PAIRED, SOAP_EFFECT_TOT>(A, depth, grid, st);
  }
}

template <typename T, int PC>
ApplyArgs<T> make_args(soap_ctx* c, const Plan& pl, const void* win, const int* nvg, void* flux, int order) {
  constexpr int R = ApplyShape<T, PC>::R, TILE = ApplyShape<T, PC>::TILE;
  const bool vec_ok = (c->P % R == 0) && (reinterpret_cast<uintptr_t>(flux) % 16 == 0);
  ApplyArgs<T> A{c->P, c->Pstride, c->con_spot_stride, c->B, pl.n_ph, pl.n_chunks, (int)((c->P + TILE - 1) / TILE),
                 pl.effect, pl.paired, pl.vg_cap, vec_ok ? 1 : 0, order,
                 (const T*)c->d_spec[0], (const T*)c->d_spec[1], (const T*)c->d_spec[2], (const T*)c->d_con_spot,
                 (const T*)c->d_con_fac, (const T*)c->d_ones, c->d_Q, static_cast<const unsigned char*>(win), nvg,
                 (T*)flux};
  return A;
}

template <typename T, int PC>
hipError_t launch_apply_pc(soap_ctx* c, const Plan& pl, const void* d_win, const int* d_nvg, void* d_flux, int depth,
                           int order, hipStream_t st) {
  const ApplyArgs<T> A = make_args<T, PC>(c, pl, d_win, d_nvg, d_flux, order);
  return pl.paired ? launch_apply_t<T, PC, true>(pl, A, depth, st) : launch_apply_t<T, PC, false>(pl, A, depth, st);
}

}  // namespace

hipError_t launch_apply(soap_ctx* c, const Plan& pl, const void* d_win, const int* d_nvg, void* d_flux) {
  return launch_apply_shape(c, pl, d_win, d_nvg, d_flux, c->tune_depth, c->tune_order, c->stream);
}

hipError_t launch_apply_shape(soap_ctx* c, const Plan& pl, const void* d_win, const int* d_nvg, void* d_flux,
                              int depth, int order, hipStream_t st) {
  const bool fp32 = c->prec == SOAP_PREC_FP32;
  if (!pc_valid(fp32, pl.pc)) return hipErrorInvalidValue;
  if (fp32)
    return pl.pc == PC_F32_WIDE ? launch_apply_pc<float, PC_F32_WIDE>(c, pl, d_win, d_nvg, d_flux, depth, order, st)
                                : launch_apply_pc<float, PC_F32>(c, pl, d_win, d_nvg, d_flux, depth, order, st);
  return pl.pc == PC_F64_WIDE ? launch_apply_pc<double, PC_F64_WIDE>(c, pl, d_win, d_nvg, d_flux, depth, order, st)
                              : launch_apply_pc<double, PC_F64>(c, pl, d_win, d_nvg, d_flux, depth, order, st);
}

// ---- batched shift-and-sum over many configurations ------------------------

namespace {

template <typename T, int PC>
hipError_t upload_t(const ApplyBatchCfg* cfgs, int n, void* d_buf, ApplyBatchGroup* g) {
  std::vector<ApplyArgs<T>> args(n);
  std::vector<int> off(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    args[i] = make_args<T, PC>(cfgs[i].c, cfgs[i].pl, cfgs[i].win, cfgs[i].nvg, cfgs[i].flux, cfgs[i].c->tune_order);
    off[i + 1] = off[i] + 8 * ((args[i].n_tiles + 7) / 8) * args[i].n_chunks;  // whole XCD rounds
  }
  g->n_cfg = n;
  g->n_items = off[n];
  g->args = d_buf;
  g->off = static_cast<unsigned char*>(d_buf) + 256 * ((sizeof(ApplyArgs<T>) * n + 255) / 256);
  hipError_t e = hipMemcpy(g->args, args.data(), sizeof(ApplyArgs<T>) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemcpy(g->off, off.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice);
}

template <typename T, int PC, bool PAIRED, int EFF>
void launch_batch_e(const ApplyBatchGroup& g, hipStream_t st) {
  const dim3 grid((unsigned)g.n_items), block(APPLY_WAVES * 64);
  const auto* a = static_cast<const ApplyArgs<T>*>(g.args);
  const int* off = static_cast<const int*>(g.off);
  if (g.depth >= 3)
    hipLaunchKernelGGL((k_apply_batch<T, PC, PAIRED, EFF, 3>), grid, block, 0, st, a, off, g.n_cfg);
  else
    hipLaunchKernelGGL((k_apply_batch<T, PC, PAIRED, EFF, 2>), grid, block, 0, st, a, off, g.n_cfg);
}

// every configuration of a batch group has the group's effect
template <typename T, int PC, bool PAIRED>
void launch_batch_t(const ApplyBatchGroup& g, hipStream_t st) {
  switch (g.effect) {
    case SOAP_EFFECT_FLUX:
      launch_batch_e<T, PC, PAIRED, SOAP_EFFECT_FLUX>(g, st);
      break;
    case SOAP_EFFECT_BCONV:
      launch_batch_e<T, PC, PAIRED, SOAP_EFFECT_BCONV>(g, st);
      break;
    default:
      launch_batch_e<T, PC, PAIRED, SOAP_EFFECT_TOT>(g, st);
      break;
  }
}

template <typename T, int PC>
void launch_batch_pc(const ApplyBatchGroup& g, hipStream_t st) {
  if (g.paired)
    launch_batch_t<T, PC, true>(g, st);
  else
    launch_batch_t<T, PC, false>(g, st);
}

}  // namespace

size_t apply_batch_bytes(int n) {
  return 256 * ((sizeof(ApplyArgs<double>) * n + 255) / 256) + sizeof(int) * (n + 1) + 256;
}

hipError_t apply_batch_upload(const ApplyBatchCfg* cfgs, int n, void* d_buf, ApplyBatchGroup* g) {
  g->fp32 = cfgs[0].c->prec == SOAP_PREC_FP32;
  g->paired = cfgs[0].pl.paired != 0;
  g->depth = cfgs[0].c->tune_depth;
  g->effect = cfgs[0].pl.effect;
  g->pc = cfgs[0].pl.pc;
  if (!pc_valid(g->fp32, g->pc)) return hipErrorInvalidValue;
  // one precision, table mode, effect, phases per chunk and depth per group
  for (int i = 1; i < n; ++i)
    if ((cfgs[i].c->prec == SOAP_PREC_FP32) != g->fp32 || (cfgs[i].pl.paired != 0) != g->paired ||
        cfgs[i].pl.effect != g->effect || cfgs[i].pl.pc != g->pc || cfgs[i].c->tune_depth != g->depth)
      return hipErrorInvalidValue;
  if (g->fp32)
    return g->pc == PC_F32_WIDE ? upload_t<float, PC_F32_WIDE>(cfgs, n, d_buf, g) : upload_t<float, PC_F32>(cfgs, n, d_buf, g);
  return g->pc == PC_F64_WIDE ? upload_t<double, PC_F64_WIDE>(cfgs, n, d_buf, g) : upload_t<double, PC_F64>(cfgs, n, d_buf, g);
}

hipError_t apply_batch_launch(const ApplyBatchGroup& g, hipStream_t st) {
  if (g.n_items <= 0) return hipSuccess;
  if (g.fp32) {
    if (g.pc == PC_F32_WIDE)
      launch_batch_pc<float, PC_F32_WIDE>(g, st);
    else
      launch_batch_pc<float, PC_F32>(g, st);
  } else {
    if (g.pc == PC_F64_WIDE)
      launch_batch_pc<double, PC_F64_WIDE>(g, st);
    else
      launch_batch_pc<double, PC_F64>(g, st);
  }
  return hipGetLastError();
}

}  // namespace soap
