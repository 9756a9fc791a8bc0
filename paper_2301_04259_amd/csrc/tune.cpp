// Tuner of the shift-and-sum kernel's shape (include/soap.h, soap_autotune):
// times every (phases per chunk, windows in flight per wave, item order)
// variant on a context's real tap lists (built once per phases-per-chunk
// value, the table layout) and keeps the fastest, with a file cache keyed by
// the shape of the work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "soap_internal.hpp"

#define SOAP_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr int kDepths[] = {2, 3};
constexpr int kOrders[] = {0, 1};

int ilog2_ceil(long long v) {
  int b = 0;
  while ((1LL << b) < v) ++b;
  return b;
}

// cache file: one entry per line, `"key": [phases per chunk, depth, order,
// apply_us],` inside a JSON object
bool cache_lookup(const char* path, const std::string& key, int* pc, int* dp, int* od, double* us) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  const std::string want = "\"" + key + "\"";
  while (std::fgets(line, sizeof line, f)) {
    const char* p = std::strstr(line, want.c_str());
    if (!p) continue;
    p = std::strchr(p + want.size(), '[');
    if (p && std::sscanf(p, "[%d , %d , %d , %lf", pc, dp, od, us) == 4) found = true;
  }
  std::fclose(f);
  return found;
}

bool cache_store(const char* path, const std::string& key, int pc, int dp, int od, double us) {
  std::vector<std::string> keep;
  if (FILE* f = std::fopen(path, "r")) {
    char line[512];
    const std::string want = "\"" + key + "\"";
    while (std::fgets(line, sizeof line, f)) {
      std::string s(line);
      while (!s.empty() && (s.back() == '\n' || s.back() == ',' || s.back() == ' ')) s.pop_back();
      if (s.empty() || s == "{" || s == "}" || s.find(want) != std::string::npos) continue;
      keep.push_back(s);
    }
    std::fclose(f);
  }
  char entry[512];
  std::snprintf(entry, sizeof entry, "  \"%s\": [%d, %d, %d, %.3f]", key.c_str(), pc, dp, od, us);
  keep.push_back(entry);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  for (size_t i = 0; i < keep.size(); ++i) std::fprintf(f, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

static int default_pc(const soap_ctx* c) { return c->prec == SOAP_PREC_FP32 ? soap::PC_F32 : soap::PC_F64; }
static int wide_pc(const soap_ctx* c) { return c->prec == SOAP_PREC_FP32 ? soap::PC_F32_WIDE : soap::PC_F64_WIDE; }

SOAP_API soap_status soap_set_apply_shape(soap_ctx* c, int32_t depth, int32_t order, int32_t phases_per_chunk) {
  if (!c) return SOAP_ERR_ARG;
  const bool d_ok = std::find(std::begin(kDepths), std::end(kDepths), depth) != std::end(kDepths);
  const bool o_ok = std::find(std::begin(kOrders), std::end(kOrders), order) != std::end(kOrders);
  const int pc = phases_per_chunk == 0 ? default_pc(c) : phases_per_chunk;
  if (!d_ok || !o_ok || !soap::pc_valid(c->prec == SOAP_PREC_FP32, pc)) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "depth must be 2 or 3, order 0 or 1 and phases_per_chunk 0, %d or %d", default_pc(c),
                  wide_pc(c));
    c->err = buf;
    return SOAP_ERR_ARG;
  }
  c->tune_depth = depth;
  c->tune_order = order;
  c->pc = pc;
  return SOAP_OK;
}

SOAP_API soap_status soap_autotune(soap_ctx* c, const soap_region* regions, int32_t n_regions,
                                   const double* phases, int32_t n_phases, int32_t effect, const char* cache_path,
                                   soap_tune* out) {
  if (!c) return SOAP_ERR_ARG;
  if (!out) {
    c->err = "out is NULL";
    return SOAP_ERR_ARG;
  }
  std::memset(out, 0, sizeof *out);
  void* tmp = nullptr;
  if (soap::dev_malloc(&tmp, (size_t)std::max(1, n_phases) * c->P * c->esize) != hipSuccess) {
    c->err = std::string("autotune: no device memory for a trial output") + soap::dev_cap_note();
    return SOAP_ERR_OOM;
  }
  const int keep_pc = c->pc;
  auto fail = [&](soap_status s, const char* msg) {
    if (msg) c->err = msg;
    if (s != SOAP_OK) c->pc = keep_pc;
    (void)hipStreamSynchronize(c->stream);
    (void)soap::dev_free(tmp);
    return s;
  };
  // one ordinary call per table layout builds this workload's tap lists (the
  // first also checks the arguments); they stay in the context's last table
  // set, which the trial launches read
  soap::Plan pl;
  auto build = [&](int pc) -> soap_status {
    c->pc = pc;
    soap_status st = soap_active_spectra(c, regions, n_regions, phases, n_phases, effect, tmp, 1);
    if (st != SOAP_OK) return st;
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
      c->err = "autotune: stream failed";
      return SOAP_ERR_HIP;
    }
    pl = soap::Plan();
    pl.n_ph = c->last_phases;
    pl.effect = c->last_effect;
    pl.paired = c->last_paired;
    pl.G = (pl.paired ? 2 : 3) * c->B;
    pl.pc = c->last_pc;
    pl.n_chunks = (pl.n_ph + pl.pc - 1) / pl.pc;
    pl.vg_cap = c->last_vg_cap;
    return SOAP_OK;
  };
  soap_status st = build(default_pc(c));
  if (st != SOAP_OK) return fail(st, nullptr);
  // key: the work's shape, with the window count of the default layout
  long long tot = 0;
  {
    soap_ctx::PrepSet& S = c->prep[c->last_prep];
    std::vector<int> nvg(pl.n_chunks);
    if (hipMemcpy(nvg.data(), S.nvg.ptr, sizeof(int) * pl.n_chunks, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(SOAP_ERR_HIP, "autotune: reading window counts failed");
    for (int v : nvg) tot += v;
  }
  char key[256];
  std::snprintf(key, sizeof key, "v4|%s|%s|P2^%d|J%d|B%d|ph2^%d|win2^%d", c->prec == SOAP_PREC_FP32 ? "f32" : "f64",
                pl.paired ? "paired" : "split", ilog2_ceil(c->P), c->J, c->B, ilog2_ceil(pl.n_ph),
                ilog2_ceil(std::max(1LL, tot / std::max(1, pl.n_chunks))));
  int cpc = 0, dp = 0, od = 0;
  double us = 0.0;
  if (cache_path && cache_lookup(cache_path, key, &cpc, &dp, &od, &us) &&
      soap_set_apply_shape(c, dp, od, cpc) == SOAP_OK) {
    out->depth = dp;
    out->order = od;
    out->phases_per_chunk = cpc;
    out->apply_us = us;
    out->from_cache = 1;
    std::snprintf(out->key, sizeof out->key, "%s", key);
    return fail(SOAP_OK, nullptr);
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(SOAP_ERR_HIP, "autotune: event creation failed");
  auto done_events = [&]() {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  };
  double best = 1e300;
  int bp = default_pc(c), bd = c->tune_depth, bo = c->tune_order, tried = 0;
  constexpr int kReps = 10;
  const int pcs[2] = {default_pc(c), wide_pc(c)};
  for (int pc : pcs) {
    if (pc != pl.pc) {
      st = build(pc);
      if (st != SOAP_OK) {
        done_events();
        return fail(st, nullptr);
      }
    }
    soap_ctx::PrepSet& S = c->prep[c->last_prep];
    for (int d : kDepths) {
      for (int o : kOrders) {
        for (int r = 0; r < 2; ++r)
          (void)soap::launch_apply_shape(c, pl, S.vg.ptr, static_cast<const int*>(S.nvg.ptr), tmp, d, o, c->stream);
        (void)hipEventRecord(e0, c->stream);
        for (int r = 0; r < kReps; ++r)
          (void)soap::launch_apply_shape(c, pl, S.vg.ptr, static_cast<const int*>(S.nvg.ptr), tmp, d, o, c->stream);
        (void)hipEventRecord(e1, c->stream);
        if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) {
          done_events();
          return fail(SOAP_ERR_HIP, "autotune: a trial launch failed");
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double t_us = 1e3 * ms / kReps;
        ++tried;
        if (t_us < best) {
          best = t_us;
          bp = pc;
          bd = d;
          bo = o;
        }
      }
    }
  }
  done_events();
  c->pc = bp;
  c->tune_depth = bd;
  c->tune_order = bo;
  out->depth = bd;
  out->order = bo;
  out->phases_per_chunk = bp;
  out->apply_us = best;
  out->n_tried = tried;
  std::snprintf(out->key, sizeof out->key, "%s", key);
  if (cache_path && !cache_store(cache_path, key, bp, bd, bo, best))
    return fail(SOAP_ERR_ARG, "autotune: cannot write the cache file");
  return fail(SOAP_OK, nullptr);
}
