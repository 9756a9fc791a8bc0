// Batched synthesis of many activity configurations of many stars
// (include/soap.h, soap_batch_*): the table kernels (region parameters,
// weights, tap lists) of every configuration run as work-list launches (one
// per kernel and precision; configurations with differential rotation get
// one launch each, on parallel branches), followed by one shift-and-sum
// launch per group of equal shape whose blocks walk the (configuration, tile,
// phase chunk) work list of its configurations; all of it is captured once
// into a HIP graph, so a run is a single graph launch with no host work per
// configuration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "soap_internal.hpp"

#define SOAP_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr int kBranches = 4;

size_t al(size_t b) { return 256 * ((b + 255) / 256); }

struct CfgPlan {
  soap_ctx* c;
  soap::Plan pl;
  int n_reg;
  size_t off_reg, off_ph, off_regcopy, off_cen, off_box, off_kfx, off_k, off_mask, off_vg, off_nvg;
  void* flux;
};

}  // namespace

struct soap_batch {
  hipStream_t launch = nullptr;                // stream the graph is launched on
  hipStream_t origin = nullptr;                // capture origin (owned)
  hipStream_t branch[kBranches] = {};          // owned
  hipEvent_t fork = nullptr, join[kBranches] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* arena = nullptr;
  int n_cfg = 0;
  int64_t n_spectra = 0;
  std::string err;
};

namespace {

void destroy_batch(soap_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (int i = 0; i < kBranches; ++i) {
    if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    if (b->branch[i]) (void)hipStreamDestroy(b->branch[i]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->origin) (void)hipStreamDestroy(b->origin);
  if (b->arena) (void)soap::dev_free(b->arena);
  delete b;
}

bool is_fin(double v) { return std::isfinite(v); }

}  // namespace

static thread_local std::string g_batch_err;

// Arena of the one-shot calls (soap_active_spectra_multi): kept between calls
// and reused under a lock, since each call waits for its stream.
struct DirectArena {
  std::mutex mu;
  void* ptr = nullptr;
  size_t bytes = 0;
  int dev = -1;
};
static DirectArena g_direct;

// Builds a batch (a graph of every configuration's work) or, with direct,
// enqueues the same launches once on hip_stream, waits for them and keeps
// nothing but the reusable arena.
static soap_status create_impl(soap_ctx* const* ctxs, int32_t n_cfg, const soap_region* regions,
                               const int32_t* region_offsets, const double* phases, const int32_t* phase_offsets,
                               int32_t effect, void* const* flux, const soap_mask* mask, double* const* ccf,
                               soap_rv* const* rv, void* hip_stream, soap_batch** out, bool direct = false) {
  auto bad = [](const std::string& m, soap_status st = SOAP_ERR_ARG) {
    g_batch_err = m;
    return st;
  };
  if (!direct && !out) return bad("out is NULL");
  if (out) *out = nullptr;
  if (!ctxs || !region_offsets || !phase_offsets || !phases || !flux) return bad("a required array is NULL");
  if (n_cfg < 1 || n_cfg > (1 << 16)) return bad("n_cfg must be in [1, 65536]");
  if (effect != SOAP_EFFECT_TOT && effect != SOAP_EFFECT_FLUX && effect != SOAP_EFFECT_BCONV)
    return bad("unknown effect");
  if (region_offsets[0] != 0 || phase_offsets[0] != 0) return bad("offsets must start at 0");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return bad("no device");
  std::vector<CfgPlan> cp(n_cfg);
  size_t arena = 0, params_bytes = 0;
  int64_t n_spec = 0;
  char msg[256];
  for (int i = 0; i < n_cfg; ++i) {
    soap_ctx* c = ctxs[i];
    if (!c || !flux[i]) return bad("a context or flux pointer is NULL");
    if (c->device != dev) return bad("every context must live on the current device");
    const int r0 = region_offsets[i], nr = region_offsets[i + 1] - r0;
    const int p0 = phase_offsets[i], np = phase_offsets[i + 1] - p0;
    if (nr < 0 || nr > soap::MAX_REGIONS) {
      std::snprintf(msg, sizeof msg, "configuration %d has %d regions (0 .. %d allowed)", i, nr, soap::MAX_REGIONS);
      return bad(msg);
    }
    if (np < 1 || np > soap::MAX_PHASES) {
      std::snprintf(msg, sizeof msg, "configuration %d has %d phases", i, np);
      return bad(msg);
    }
    if (nr > 0 && !regions) return bad("regions is NULL");
    bool unit = true;
    double cmax = 1.0;
    for (int r = r0; r < r0 + nr; ++r) {
      const soap_region& R = regions[r];
      if ((R.type != SOAP_SPOT && R.type != SOAP_FACULA) || !is_fin(R.lat_deg) || R.lat_deg < -90.0 ||
          R.lat_deg > 90.0 || !is_fin(R.lon_deg) || !(R.radius > 0.0 && R.radius < 1.0) || !is_fin(R.contrast) ||
          !(R.contrast > 0.0) || (effect != SOAP_EFFECT_FLUX && !c->has_type[R.type])) {
        std::snprintf(msg, sizeof msg, "configuration %d: region %d is invalid for its star", i, r - r0);
        return bad(msg);
      }
      unit = unit && R.contrast == 1.0;
      cmax = std::max(cmax, R.contrast);
    }
    for (int p = p0; p < p0 + np; ++p)
      if (!is_fin(phases[p])) return bad("a phase is not finite");
    CfgPlan& q = cp[i];
    q.c = c;
    q.n_reg = nr;
    q.flux = flux[i];
    soap::Plan& pl = q.pl;
    pl.n_ph = np;
    pl.effect = effect;
    pl.paired = (c->cmode != SOAP_CONTRAST_SCALAR || effect == SOAP_EFFECT_BCONV || unit) ? 1 : 0;
    if (!pl.paired && !(c->disk_weight * cmax < soap::FX_RANGE)) {
      // split tables scale the active rows by the contrasts: the fixed-point
      // tap sums hold |x| < 16
      std::snprintf(msg, sizeof msg, "configuration %d: disk weight x contrast reaches the fixed-point range", i);
      return bad(msg, SOAP_ERR_UNSUPPORTED);
    }
    pl.G = (pl.paired ? 2 : 3) * c->B;
    pl.n_slabs = (c->N + soap::SLAB_COLS - 1) / soap::SLAB_COLS;
    pl.pc = c->pc;
    pl.n_chunks = (np + pl.pc - 1) / pl.pc;
    pl.vg_cap = pl.G * ((c->J + soap::APPLY_JW - 1) / soap::APPLY_JW);
    const size_t GJ = (size_t)pl.G * c->J;
    auto take = [&](size_t bytes) {
      const size_t o = arena;
      arena += al(std::max<size_t>(bytes, 1));
      return o;
    };
    // regions and phases of every configuration form the arena's first
    // section (one upload); the other offsets are shifted past it below
    auto ptake = [&](size_t bytes) {
      const size_t o = params_bytes;
      params_bytes += al(std::max<size_t>(bytes, 1));
      return o;
    };
    q.off_reg = ptake(sizeof(soap::Region) * std::max(1, nr));
    q.off_ph = ptake(sizeof(double) * np);
    q.off_regcopy = take(sizeof(soap::Region) * std::max(1, nr));
    q.off_cen = take(sizeof(double4) * (size_t)np * std::max(1, nr));
    q.off_box = take(sizeof(int4) * (size_t)np);
    q.off_kfx = take(sizeof(unsigned long long) * (size_t)np * GJ);
    q.off_k = take(sizeof(double) * (size_t)np * GJ);
    q.off_mask = take(sizeof(unsigned long long) * (size_t)np * pl.G);
    q.off_vg = take((size_t)soap::win_bytes(pl.pc, (int)c->esize) * pl.n_chunks * pl.vg_cap);
    q.off_nvg = take(sizeof(int) * (size_t)pl.n_chunks);
    n_spec += np;
  }
  for (CfgPlan& q : cp) {
    size_t* offs[] = {&q.off_regcopy, &q.off_cen, &q.off_box, &q.off_kfx, &q.off_k, &q.off_mask, &q.off_vg, &q.off_nvg};
    for (size_t* o : offs) *o += params_bytes;
  }
  arena += params_bytes;
  // the shift-and-sum runs as one launch per (precision, table mode, phases
  // per chunk, windows in flight) over every configuration's (tile, chunk)
  // items, in order of first appearance
  std::vector<std::vector<int>> groups;
  {
    std::vector<long long> keys;
    for (int i = 0; i < n_cfg; ++i) {
      const soap_ctx* c = cp[i].c;
      const long long k = ((long long)(c->prec == SOAP_PREC_FP32) << 40) | ((long long)cp[i].pl.paired << 32) |
                          ((long long)cp[i].pl.pc << 8) | (long long)c->tune_depth;
      size_t g = 0;
      while (g < keys.size() && keys[g] != k) ++g;
      if (g == keys.size()) {
        keys.push_back(k);
        groups.emplace_back();
      }
      groups[g].push_back(i);
    }
  }
  const int n_groups = (int)groups.size();
  std::vector<size_t> group_off(n_groups, 0);
  for (int g = 0; g < n_groups; ++g) {
    group_off[g] = arena;
    arena += al(soap::apply_batch_bytes((int)groups[g].size()));
  }
  // the table kernels of configurations with solid-body rotation run as
  // work-list launches; those with differential rotation keep one launch
  // each, spread over the branches
  std::vector<int> listed, single;
  for (int i = 0; i < n_cfg; ++i) (cp[i].c->diff_rot != 0.0 ? single : listed).push_back(i);
  // host copies of every configuration's regions (kernel layout)
  std::vector<std::vector<soap::Region>> hregs(n_cfg);
  for (int i = 0; i < n_cfg; ++i) {
    const int r0 = region_offsets[i];
    hregs[i].assign(std::max(1, cp[i].n_reg), soap::Region{});
    for (int r = 0; r < cp[i].n_reg; ++r) {
      const soap_region& R = regions[r0 + r];
      hregs[i][r] = soap::Region{R.type, 0, R.lat_deg, R.lon_deg, R.radius, R.contrast};
    }
  }
  // work-list entries (device pointers filled in once the arena exists)
  std::vector<soap::TableBatchCfg> tc;
  for (int i : listed)
    tc.push_back(soap::TableBatchCfg{cp[i].c, cp[i].pl, nullptr, cp[i].n_reg, std::max(1, cp[i].n_reg), nullptr,
                                     soap::WeightsOut{}, hregs[i].data(), phases + phase_offsets[i]});
  const size_t table_off = arena;
  if (!listed.empty()) arena += al(soap::table_batch_bytes(tc.data(), (int)tc.size()));
  // CCF + fit stage: each distinct context's mask tables are copied into the
  // arena (the batch must not depend on a later mask of the context), and
  // every configuration gets its line-block partials (and CCF rows when the
  // caller gives none)
  std::vector<soap_ctx*> uctx;           // distinct contexts
  std::vector<size_t> tab_off;           // their table copies
  std::vector<int> ucfg(n_cfg, -1);      // configuration -> distinct context
  std::vector<size_t> part_off(n_cfg, 0), ccf_off(n_cfg, 0);
  std::vector<std::vector<int>> ccf_groups;  // configurations per CCF layout
  std::vector<size_t> ccf_group_off;
  if (mask) {
    for (int i = 0; i < n_cfg; ++i) {
      soap_ctx* c = cp[i].c;
      size_t u = 0;
      while (u < uctx.size() && uctx[u] != c) ++u;
      if (u == uctx.size()) {
        const soap_status ms = soap::ctx_set_mask(c, mask);
        if (ms != SOAP_OK) return bad("configuration " + std::to_string(i) + ": " + c->err, ms);
        uctx.push_back(c);
        tab_off.push_back(arena);
        arena += al(c->mask_blob_bytes);
      }
      ucfg[i] = (int)u;
      const size_t nlb = (size_t)soap::ccf_line_blocks(c->ccf_nl);
      part_off[i] = arena;
      arena += al(c->esize * nlb * (size_t)cp[i].pl.n_ph * c->mask_nv);
      if (!ccf || !ccf[i]) {
        ccf_off[i] = arena;
        arena += al(sizeof(double) * (size_t)cp[i].pl.n_ph * c->mask_nv);
      }
    }
    // one work-list CCF + fit launch pair per mask layout (float type,
    // pixels per hole, stage width)
    std::vector<soap::CcfPlan> shape(uctx.size());
    for (size_t u = 0; u < uctx.size(); ++u) shape[u] = soap::ccf_plan(uctx[u], uctx[u]->ccf_nl, nullptr);
    for (int i = 0; i < n_cfg; ++i) {
      const soap::CcfPlan& q = shape[ucfg[i]];
      size_t g = 0;
      while (g < ccf_groups.size() && !soap::ccf_same_layout(shape[ucfg[ccf_groups[g][0]]], q)) ++g;
      if (g == ccf_groups.size()) ccf_groups.emplace_back();
      ccf_groups[g].push_back(i);
    }
    for (const auto& grp : ccf_groups) {
      std::vector<soap::CcfPlan> pl;
      std::vector<int64_t> ns;
      for (int i : grp) {
        pl.push_back(shape[ucfg[i]]);
        ns.push_back(cp[i].pl.n_ph);
      }
      ccf_group_off.push_back(arena);
      arena += al(soap::ccf_batch_bytes(pl.data(), ns.data(), (int)grp.size()));
    }
  }

  soap_batch* b = new soap_batch;
  b->n_cfg = n_cfg;
  b->n_spectra = n_spec;
  b->launch = static_cast<hipStream_t>(hip_stream);
  auto fail = [&](const char* what, hipError_t e) {
    g_batch_err = std::string(what) + ": " + hipGetErrorString(e) +
                  (e == hipErrorOutOfMemory ? soap::dev_cap_note() : "");
    destroy_batch(b);
    return (e == hipErrorOutOfMemory) ? SOAP_ERR_OOM : SOAP_ERR_HIP;
  };
  hipError_t e;
  std::unique_lock<std::mutex> direct_lock;
  unsigned char* A = nullptr;
  if (direct) {
    direct_lock = std::unique_lock<std::mutex>(g_direct.mu);
    if (g_direct.bytes < arena || g_direct.dev != dev) {
      if (g_direct.ptr) (void)soap::dev_free(g_direct.ptr);
      g_direct.ptr = nullptr;
      g_direct.bytes = 0;
      if ((e = soap::dev_malloc(&g_direct.ptr, arena)) != hipSuccess) return fail("hipMalloc", e);
      g_direct.bytes = arena;
      g_direct.dev = dev;
    }
    A = static_cast<unsigned char*>(g_direct.ptr);
  } else {
    if ((e = soap::dev_malloc(&b->arena, arena)) != hipSuccess) return fail("hipMalloc", e);
    A = static_cast<unsigned char*>(b->arena);
  }
  // tap accumulators start at zero (each run's tap-list kernel clears them
  // again after reading); parameters are uploaded once
  if ((e = hipMemset(A, 0, arena)) != hipSuccess) return fail("hipMemset", e);
  {
    std::vector<unsigned char> hp(params_bytes, 0);
    for (int i = 0; i < n_cfg; ++i) {
      const CfgPlan& q = cp[i];
      const std::vector<soap::Region>& hr = hregs[i];
      std::memcpy(hp.data() + q.off_reg, hr.data(), sizeof(soap::Region) * hr.size());
      std::memcpy(hp.data() + q.off_ph, phases + phase_offsets[i], sizeof(double) * q.pl.n_ph);
    }
    if ((e = hipMemcpy(A, hp.data(), params_bytes, hipMemcpyHostToDevice)) != hipSuccess) return fail("hipMemcpy", e);
  }
  std::vector<soap::CcfPlan> cplan(uctx.size());
  for (size_t u = 0; u < uctx.size(); ++u) {
    soap_ctx* c = uctx[u];
    // the mask upload is enqueued on the context's stream
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return fail("context stream", e);
    if ((e = hipMemcpy(A + tab_off[u], c->ws_mask.ptr, c->mask_blob_bytes, hipMemcpyDeviceToDevice)) != hipSuccess)
      return fail("copying the mask tables", e);
    cplan[u] = soap::ccf_plan(c, c->ccf_nl, A + tab_off[u]);
  }
  std::vector<soap::CcfBatch> cbat(ccf_groups.size());
  for (size_t g = 0; g < ccf_groups.size(); ++g) {
    std::vector<soap::CcfPlan> pl;
    std::vector<soap::CcfBatchSet> sets;
    for (int i : ccf_groups[g]) {
      pl.push_back(cplan[ucfg[i]]);
      soap::CcfBatchSet cs{};
      cs.flux = cp[i].flux;
      cs.part = A + part_off[i];
      cs.ccf = (ccf && ccf[i]) ? ccf[i] : reinterpret_cast<double*>(A + ccf_off[i]);
      cs.rv = rv ? rv[i] : nullptr;
      cs.n_spec = cp[i].pl.n_ph;
      sets.push_back(cs);
    }
    if ((e = soap::ccf_batch_upload(pl.data(), sets.data(), (int)sets.size(), A + ccf_group_off[g], &cbat[g])) !=
        hipSuccess)
      return fail("uploading the CCF work lists", e);
  }
  std::vector<soap::ApplyBatchGroup> ag(n_groups);
  for (int g = 0; g < n_groups; ++g) {
    std::vector<soap::ApplyBatchCfg> ac;
    for (int i : groups[g])
      ac.push_back(soap::ApplyBatchCfg{cp[i].c, cp[i].pl, A + cp[i].off_vg,
                                       reinterpret_cast<const int*>(A + cp[i].off_nvg), cp[i].flux});
    if ((e = soap::apply_batch_upload(ac.data(), (int)ac.size(), A + group_off[g], &ag[g])) != hipSuccess)
      return fail("uploading the shift-and-sum work list", e);
  }
  auto outs_of = [&](const CfgPlan& q) {
    soap::WeightsOut wo;
    wo.reg = reinterpret_cast<soap::Region*>(A + q.off_regcopy);
    wo.pj = nullptr;
    wo.cen = reinterpret_cast<double4*>(A + q.off_cen);
    wo.box = reinterpret_cast<int4*>(A + q.off_box);
    wo.Kfx = reinterpret_cast<unsigned long long*>(A + q.off_kfx);
    wo.K = reinterpret_cast<double*>(A + q.off_k);
    wo.mask = reinterpret_cast<unsigned long long*>(A + q.off_mask);
    wo.wins = A + q.off_vg;
    wo.nvg = reinterpret_cast<int*>(A + q.off_nvg);
    return wo;
  };
  soap::TableBatch tb;
  if (!listed.empty()) {
    for (size_t u = 0; u < listed.size(); ++u) {
      const CfgPlan& q = cp[listed[u]];
      tc[u].d_reg = reinterpret_cast<const soap::Region*>(A + q.off_reg);
      tc[u].d_ph = reinterpret_cast<const double*>(A + q.off_ph);
      tc[u].o = outs_of(q);
    }
    if ((e = soap::table_batch_upload(tc.data(), (int)tc.size(), A + table_off, &tb)) != hipSuccess)
      return fail("uploading the table work lists", e);
  }
  // The tables the launches read (local spectra, contrast rows, Q) are
  // written only by soap_grid_init, which waits for its work before it
  // returns; a batch graph, replayed later, also waits here once for every
  // distinct context's streams.  The one-shot call does not wait (per
  // configuration that cost more than its kernels).
  if (!direct) {
    std::vector<soap_ctx*> seen;
    for (int i = 0; i < n_cfg; ++i) {
      soap_ctx* c = cp[i].c;
      if (std::find(seen.begin(), seen.end(), c) != seen.end()) continue;
      seen.push_back(c);
      if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return fail("context stream", e);
      if ((e = hipStreamSynchronize(c->side)) != hipSuccess) return fail("context stream", e);
    }
  }
  // Every launch of one run: with fork_join, work per configuration spreads
  // over the branch streams (forked from and joined to org); without, it all
  // goes on org in order.
  auto enqueue = [&](hipStream_t org, bool fork_join) -> hipError_t {
    auto lane = [&](size_t u) { return fork_join ? b->branch[u % kBranches] : org; };
    hipError_t ce = hipSuccess;
    if (fork_join) {
      ce = hipEventRecord(b->fork, org);
      for (int k = 0; k < kBranches && ce == hipSuccess; ++k) ce = hipStreamWaitEvent(b->branch[k], b->fork, 0);
    }
    for (size_t u = 0; u < single.size() && ce == hipSuccess; ++u) {
      const CfgPlan& q = cp[single[u]];
      const soap::WeightsOut wo = outs_of(q);
      ce = soap::launch_weights(q.c, q.pl, reinterpret_cast<const soap::Region*>(A + q.off_reg), q.n_reg,
                                std::max(1, q.n_reg), reinterpret_cast<const double*>(A + q.off_ph), nullptr, wo,
                                lane(u));
      if (ce == hipSuccess) ce = soap::launch_finish(q.c, q.pl, wo, lane(u));
    }
    if (ce == hipSuccess && !listed.empty()) ce = soap::table_batch_launch(tb, org);
    if (fork_join)
      for (int k = 0; k < kBranches && ce == hipSuccess; ++k) {
        ce = hipEventRecord(b->join[k], b->branch[k]);
        if (ce == hipSuccess) ce = hipStreamWaitEvent(org, b->join[k], 0);
      }
    for (int g = 0; g < n_groups && ce == hipSuccess; ++g) ce = soap::apply_batch_launch(ag[g], org);
    // CCF and fit of every configuration's spectra: one work-list pair per
    // mask layout
    for (size_t g = 0; g < cbat.size() && ce == hipSuccess; ++g) ce = soap::ccf_batch_launch(cbat[g], org);
    return ce;
  };
  if (direct) {
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipError_t ce = enqueue(st, false);
    const hipError_t se = hipStreamSynchronize(st);
    if (ce != hipSuccess) return fail("enqueueing the configurations", ce);
    if (se != hipSuccess) return fail("hipStreamSynchronize", se);
    destroy_batch(b);
    return SOAP_OK;
  }
  if ((e = hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking)) != hipSuccess) return fail("stream", e);
  for (int k = 0; k < kBranches; ++k) {
    if ((e = hipStreamCreateWithFlags(&b->branch[k], hipStreamNonBlocking)) != hipSuccess) return fail("stream", e);
    if ((e = hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming)) != hipSuccess) return fail("event", e);
  }
  if ((e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) != hipSuccess) return fail("event", e);
  if ((e = hipStreamBeginCapture(b->origin, hipStreamCaptureModeRelaxed)) != hipSuccess) return fail("capture", e);
  const hipError_t ce = enqueue(b->origin, true);
  e = hipStreamEndCapture(b->origin, &b->graph);
  if (ce != hipSuccess) return fail("capturing the batch", ce);
  if (e != hipSuccess) return fail("hipStreamEndCapture", e);
  if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
    return fail("hipGraphInstantiate", e);
  *out = b;
  return SOAP_OK;
}

SOAP_API soap_status soap_batch_create(soap_ctx* const* ctxs, int32_t n_cfg, const soap_region* regions,
                                       const int32_t* region_offsets, const double* phases,
                                       const int32_t* phase_offsets, int32_t effect, void* const* flux,
                                       void* hip_stream, soap_batch** out) {
  return create_impl(ctxs, n_cfg, regions, region_offsets, phases, phase_offsets, effect, flux, nullptr, nullptr,
                     nullptr, hip_stream, out);
}

SOAP_API soap_status soap_batch_create_rv(soap_ctx* const* ctxs, int32_t n_cfg, const soap_region* regions,
                                          const int32_t* region_offsets, const double* phases,
                                          const int32_t* phase_offsets, int32_t effect, void* const* flux,
                                          const soap_mask* mask, double* const* ccf, soap_rv* const* rv,
                                          void* hip_stream, soap_batch** out) {
  if (!mask) {
    if (out) *out = nullptr;
    g_batch_err = "mask is NULL";
    return SOAP_ERR_ARG;
  }
  return create_impl(ctxs, n_cfg, regions, region_offsets, phases, phase_offsets, effect, flux, mask, ccf, rv,
                     hip_stream, out);
}

SOAP_API soap_status soap_active_spectra_multi(soap_ctx* const* ctxs, int32_t n_cfg, const soap_region* regions,
                                               const int32_t* region_offsets, const double* phases,
                                               const int32_t* phase_offsets, int32_t effect, void* const* flux,
                                               void* hip_stream) {
  return create_impl(ctxs, n_cfg, regions, region_offsets, phases, phase_offsets, effect, flux, nullptr, nullptr,
                     nullptr, hip_stream, nullptr, true);
}

SOAP_API soap_status soap_batch_run(soap_batch* b) {
  if (!b) return SOAP_ERR_ARG;
  const hipError_t e = hipGraphLaunch(b->exec, b->launch);
  if (e != hipSuccess) {
    b->err = std::string("hipGraphLaunch: ") + hipGetErrorString(e);
    return SOAP_ERR_HIP;
  }
  return SOAP_OK;
}

SOAP_API int64_t soap_batch_n_spectra(const soap_batch* b) { return b ? b->n_spectra : -1; }

SOAP_API const char* soap_batch_last_error(const soap_batch* b) {
  return b ? b->err.c_str() : g_batch_err.c_str();
}

SOAP_API void soap_batch_destroy(soap_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->launch);
  destroy_batch(b);
}
