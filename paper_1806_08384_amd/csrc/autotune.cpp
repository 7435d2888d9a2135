// autotune.cpp -- offline search of launch configurations for the scan and
// batch kernels, keyed by program class and table size: workgroup size and
// number of workgroups, then (scans) cached or nontemporal column loads,
// tiles per wave step and the LDS staging limit, (batches) rows per lane of
// the lookup-table kernel -- one knob at a time from the fastest shape.
// The result feeds the launch lookup of every later call on the context and
// can be saved to / loaded from a file.
// Tuning launches the real kernels on the real table, so it belongs before
// serving, never on its latency path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "runtime.h"

using namespace sel;
using namespace selrt;

namespace {

struct Candidate {
  uint32_t block, grid;
};

// Launch shapes to time: for a batch (bp != nullptr) the workgroup sizes
// whose LDS fits the plan.
std::vector<Candidate> candidates(sel_ctx* ctx, int occ_mode, const BatchPlan* bp) {
  std::vector<Candidate> c;
  const bool batch = bp != nullptr;
  for (uint32_t block : {64u, 128u, 256u, 512u, kBatchBlock}) {
    if (block > 256 && !batch) continue;   // the scan kernels take at most 256
    if (batch && bp->lds_bytes(block) > kLdsPerCu) continue;
    int occ = 0;
    const int e = batch ? sel_batch_occupancy(block, bp->lds_bytes(block), &occ) : sel_scan_occupancy(occ_mode, block, &occ);
    if (e != 0 || occ < 1) occ = 1;
    const int max_waves = occ * (int)(block / kWave);
    for (int waves : {4, 8, 12, 16, 20, 24, 32}) {
      if (waves > max_waves) break;
      const uint32_t per_cu = (uint32_t)waves / (block / kWave);
      if (per_cu == 0) continue;
      c.push_back({block, per_cu * ctx->num_cus});
    }
  }
  return c;
}

template <class Launch>
sel_status time_candidates(sel_ctx* ctx, const std::vector<Candidate>& cands, uint32_t reps,
                           Launch launch, Candidate& best, double& best_ms) {
  hipEvent_t a, b;
  HIP_TRY(ctx, hipEventCreate(&a), "hipEventCreate");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return set_err(ctx, SEL_E_DEVICE, "hipEventCreate");
  }
  best_ms = 1e30;
  sel_status st = SEL_OK;
  for (const Candidate& c : cands) {
    if (launch(c) != 0) { st = set_err(ctx, SEL_E_DEVICE, "launch failed while tuning"); break; }
    std::vector<float> t;
    for (uint32_t r = 0; r < reps; ++r) {
      (void)hipEventRecord(a, ctx->stream);
      const int e = launch(c);
      (void)hipEventRecord(b, ctx->stream);
      if (e != 0 || hipEventSynchronize(b) != hipSuccess) {
        st = set_err(ctx, SEL_E_DEVICE, "launch failed while tuning");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      t.push_back(ms);
    }
    if (st != SEL_OK) break;
    std::sort(t.begin(), t.end());
    const double med = t[t.size() / 2];
    if (med < best_ms) {
      best_ms = med;
      best = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return st;
}

}  // namespace

extern "C" {

sel_status sel_autotune(sel_ctx* ctx, const sel_table* table, const sel_program* prog, int with_mask,
                        uint32_t reps, sel_launch* best, double* best_ms) {
  if (!ctx || !table || !prog) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  if (prog->table != table) return set_err(ctx, SEL_E_INVALID, "program is bound to another table");
  if (reps == 0) reps = 5;
  DeviceGuard g(ctx->device);
  const int mode = with_mask ? M_MASK : M_COUNT;
  const uint64_t ntiles = ntiles_of(table->nrows);
  ScanArgs a{};
  a.prog = prog->dcode;
  a.nins = prog->nins;
  set_stage(a, prog);
  a.nrows = table->nrows;
  a.ntiles = ntiles;
  a.out = ctx->dout;
  a.slot = ctx->slot;
  if (with_mask) {
    const RowidScratch L(ntiles);
    sel_status st = ensure_scratch(ctx, L.total());
    if (st != SEL_OK) return st;
    a.mask = (uint32_t*)ctx->scratch;
    a.tile_counts = (uint32_t*)((char*)ctx->scratch + L.mask);
    a.tile_lanes = (uint64_t*)((char*)ctx->scratch + L.mask + 2 * L.counts + 2 * L.chunk);
  }
  Candidate b{256, 0};
  double ms = 0;
  const uint64_t need_waves = std::max<uint64_t>(1, ntiles);
  sel_launch cfg = kDefaultLaunch;
  auto launch_with = [&](const sel_launch& c) {
    ScanArgs x = a;
    x.cached = c.cached;
    x.tiles_per_step = c.tiles_per_step ? c.tiles_per_step : 1;
    limit_stage(x, prog->stage_end, c.stage_words);
    const uint64_t need = (need_waves + c.block / kWave - 1) / (c.block / kWave);
    return sel_launch_scan(mode, x, (uint32_t)std::min<uint64_t>(c.grid, need), c.block, ctx->stream);
  };
  // the launch shape with the default knobs
  sel_status st = time_candidates(ctx, candidates(ctx, mode, nullptr), reps, [&](const Candidate& c) {
    sel_launch l = cfg;
    l.block = c.block;
    l.grid = c.grid;
    return launch_with(l);
  }, b, ms);
  if (st != SEL_OK) return st;
  cfg.block = b.block;
  cfg.grid = b.grid;
  // then each knob in turn, the others at their best so far
  auto knob = [&](uint32_t sel_launch::*field, std::initializer_list<uint32_t> values) -> sel_status {
    std::vector<Candidate> cs;
    for (uint32_t v : values) cs.push_back({v, 0});   // block carries the value
    Candidate kb{cfg.*field, 0};
    double kms = 0;
    const sel_status s = time_candidates(ctx, cs, reps, [&](const Candidate& c) {
      sel_launch l = cfg;
      l.*field = c.block;
      return launch_with(l);
    }, kb, kms);
    if (s == SEL_OK) {
      cfg.*field = kb.block;
      ms = kms;
    }
    return s;
  };
  if ((st = knob(&sel_launch::cached, {0u, 1u})) != SEL_OK) return st;
  if ((st = knob(&sel_launch::tiles_per_step, {1u, 2u, 4u})) != SEL_OK) return st;
  if (prog->nstage && (st = knob(&sel_launch::stage_words, {0u, 2048u, 1u})) != SEL_OK) return st;
  ctx->tune[tune_key(mode, prog->tune_class, ntiles)] = cfg;
  if (best) *best = cfg;
  if (best_ms) *best_ms = ms;
  return SEL_OK;
}

sel_status sel_autotune_batch(sel_ctx* ctx, uint32_t n, const sel_table* const* tables,
                              const sel_program* const* progs, uint32_t reps, sel_launch* best,
                              double* best_ms) {
  if (!ctx) return SEL_E_INVALID;
  if (reps == 0) reps = 3;
  // time each candidate through the eager batch call with a fixed shape
  const sel_launch saved = ctx->launch;
  const bool saved_fixed = ctx->launch_fixed;
  std::vector<uint64_t> out(n ? n : 1);
  BatchPlan bp;
  sel_status pst = plan_batch(ctx, n, tables, progs, bp);
  if (pst != SEL_OK) return pst;
  const uint64_t total_tiles = bp.total_tiles;
  DeviceGuard g(ctx->device);
  Candidate b{256, 0};
  double ms = 0;
  sel_launch cfg = kDefaultLaunch;
  sel_status st = time_candidates(ctx, candidates(ctx, 0, &bp), reps, [&](const Candidate& c) {
    ctx->launch = cfg;
    ctx->launch.block = c.block;
    ctx->launch.grid = c.grid;
    ctx->launch_fixed = true;
    return (int)sel_count_batch(ctx, n, tables, progs, out.data()) == SEL_OK ? 0 : 1;
  }, b, ms);
  cfg.block = b.block;
  cfg.grid = b.grid;
  // the lookup-table kernel's rows per lane, if the plan uses that kernel
  if (st == SEL_OK && !bp.lut.empty()) {
    Candidate rb{8, 0};
    double rms = 0;
    st = time_candidates(ctx, {{8, 0}, {4, 0}}, reps, [&](const Candidate& c) {
      ctx->launch = cfg;
      ctx->launch.rows_per_lane = c.block;
      ctx->launch_fixed = true;
      return (int)sel_count_batch(ctx, n, tables, progs, out.data()) == SEL_OK ? 0 : 1;
    }, rb, rms);
    if (st == SEL_OK) {
      cfg.rows_per_lane = rb.block;
      ms = rms;
    }
  }
  ctx->launch = saved;
  ctx->launch_fixed = saved_fixed;
  if (st != SEL_OK) return st;
  ctx->tune[tune_key(TK_BATCH, batch_class(n), total_tiles)] = cfg;
  if (best) *best = cfg;
  if (best_ms) *best_ms = ms;
  return SEL_OK;
}

// One line per entry: "key block grid cached tiles_per_step stage_words
// rows_per_lane".
sel_status sel_tune_save(const sel_ctx* ctx, const char* path) {
  if (!ctx || !path) return SEL_E_INVALID;
  FILE* f = std::fopen(path, "w");
  if (!f) return set_err(const_cast<sel_ctx*>(ctx), SEL_E_INVALID, std::string("cannot write ") + path);
  std::fprintf(f, "# libsel launch tuning: key block grid (device with %u CUs)\n", ctx->num_cus);
  for (const auto& kv : ctx->tune)
    std::fprintf(f, "%llu %u %u %u %u %u %u\n", (unsigned long long)kv.first, kv.second.block, kv.second.grid,
                 kv.second.cached, kv.second.tiles_per_step, kv.second.stage_words, kv.second.rows_per_lane);
  std::fclose(f);
  return SEL_OK;
}

sel_status sel_tune_load(sel_ctx* ctx, const char* path) {
  if (!ctx || !path) return SEL_E_INVALID;
  FILE* f = std::fopen(path, "r");
  if (!f) return set_err(ctx, SEL_E_INVALID, std::string("cannot read ") + path);
  char line[256];
  unsigned cus = 0;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') {
      std::sscanf(line, "# libsel launch tuning: key block grid (device with %u CUs)", &cus);
      continue;
    }
    unsigned long long key;
    unsigned block, grid, cached = 0, tps = 1, stage = 0, rows = 0;
    const int nf = std::sscanf(line, "%llu %u %u %u %u %u %u", &key, &block, &grid, &cached, &tps, &stage, &rows);
    if (nf != 3 && nf != 7) continue;
    if (cached > 1 || tps == 0 || tps == 3 || tps > 4 || (rows != 0 && rows != 4 && rows != 8)) continue;
    // 512 and kBatchBlock only for the batch kernel (the scan kernels take
    // at most 256)
    const bool batch_key = (key & 0xFull) == (unsigned long long)TK_BATCH;
    if (block != 64 && block != 128 && block != 256 &&
        !((block == 512 || block == kBatchBlock) && batch_key)) continue;
    if (cus && cus != ctx->num_cus) grid = (uint32_t)((uint64_t)grid * ctx->num_cus / cus);
    ctx->tune[key] = sel_launch{block, grid, cached, tps, stage, rows};
  }
  std::fclose(f);
  return SEL_OK;
}

uint32_t sel_tune_entries(const sel_ctx* ctx) { return ctx ? (uint32_t)ctx->tune.size() : 0; }

}  // extern "C"
