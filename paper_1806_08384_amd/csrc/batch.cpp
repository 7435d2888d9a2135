// batch.cpp -- many candidate predicates counted in one launch (k_batch),
// once eagerly (sel_count_batch) or as a captured, replayable HIP graph
// (sel_batch_*).  Algorithm 1 computes one exact count per candidate
// relation in its loop over the queue of relations; a batch runs all of
// them, over tables of uneven size, in a single persistent launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "runtime.h"

using namespace sel;
using namespace selrt;

struct sel_batch {
  sel_ctx* ctx = nullptr;
  uint32_t n = 0;
  std::vector<const sel_table*> tabs;         // per caller index
  std::vector<const sel_program*> slot_prog;  // per caller index
  BatchPlan plan;
  void* dev = nullptr;                        // descriptors | acc | out | slot | tables
  size_t desc_cap = 0, gtab_cap = 0;
  uint32_t* d_gtab = nullptr;
  const TableBuild* d_builds = nullptr;       // as captured
  uint32_t nbuilds = 0;
  uint64_t table_entries = 0;
  unsigned long long* d_acc = nullptr;
  unsigned long long* d_out = nullptr;
  DevSlot* d_slot = nullptr;
  unsigned long long* h_out = nullptr;        // pinned
  hipStream_t stream = nullptr;
  hipEvent_t ready = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchArgs args{};                           // as captured
  LutArgs largs{};                            // as captured
  uint32_t lut_grid = 0, lut_block = 0, lut_lds = 0;
  uint32_t grid = 0, block = 256, lds = 0;
};

namespace selrt {

// Validate the (table, program) pairs and plan one pass list per distinct
// table (first-use order); accumulator line i belongs to pair i.
sel_status plan_batch(sel_ctx* ctx, uint32_t n, const sel_table* const* tables,
                const sel_program* const* progs, BatchPlan& bp) {
  if (n == 0 || n > (uint32_t)kBatchMaxProgs)
    return set_err(ctx, SEL_E_INVALID, "batch size must be 1..1024");
  if (!tables || !progs) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  std::vector<const sel_table*> distinct;
  for (uint32_t i = 0; i < n; ++i) {
    if (!tables[i] || !progs[i]) return set_err(ctx, SEL_E_INVALID, "NULL table or program");
    if (progs[i]->table != tables[i])
      return set_err(ctx, SEL_E_INVALID, "program " + std::to_string(i) + " is bound to another table");
    if (batch_slots_alone(progs[i]) > kBatchMaxSlots)
      return set_err(ctx, SEL_E_INVALID, "program " + std::to_string(i) + " has too many leaves to batch");
    if (std::find(distinct.begin(), distinct.end(), tables[i]) == distinct.end())
      distinct.push_back(tables[i]);
  }
  bp.clear();
  bp.allow_lut = true;   // the lookup-table kernel for the programs it can express
  std::vector<const sel_program*> ps;
  std::vector<uint32_t> acc;
  for (const sel_table* t : distinct) {
    ps.clear();
    acc.clear();
    for (uint32_t i = 0; i < n; ++i) {
      if (tables[i] != t) continue;
      ps.push_back(progs[i]);
      acc.push_back(i);
    }
    bp.add(t, 0, t->nrows, ps.data(), acc.data(), (uint32_t)ps.size());
  }
  bp.num_cus = ctx->num_cus;
  return SEL_OK;
}

}  // namespace selrt

namespace {

// Launch shape of a batch: fixed by the caller, else tuned for this
// (program count, size) class, else as many workgroups of the plan's
// default size as fit a CU (registers and the plan's LDS), at most 16 waves
// per CU.  A block whose LDS would not fit the plan falls back to 512.
void batch_shape(sel_ctx* ctx, uint32_t nprogs, const BatchPlan& bp, uint32_t& grid,
                 uint32_t& block) {
  block = bp.default_block();
  uint64_t g = 0;
  uint32_t rows = 0;
  if (ctx->launch_fixed) {
    block = ctx->launch.block;
    g = ctx->launch.grid;
    rows = ctx->launch.rows_per_lane;
  } else {
    auto it = ctx->tune.find(tune_key(TK_BATCH, batch_class(nprogs), bp.total_tiles));
    if (it != ctx->tune.end()) {
      block = it->second.block;
      g = it->second.grid;
      rows = it->second.rows_per_lane;
    }
  }
  bp.lut_rows = rows == 4 ? 4u : 8u;
  if (bp.lds_bytes(block) > kLdsPerCu) {
    block = 512;
    g = 0;
  }
  if (g == 0) {
    int occ = 1;
    if (sel_batch_occupancy(block, bp.lds_bytes(block), &occ) != 0 || occ < 1) occ = 1;
    g = (uint64_t)std::min(occ, (int)(16 * 64 / block)) * ctx->num_cus;
  }
  const uint64_t need = std::max<uint64_t>(1, (bp.total_tiles + block / 64 - 1) / (block / 64));
  grid = (uint32_t)std::min(g, need);
}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace after the descriptors: accumulator lines, counts, slot.
size_t tail_bytes(uint32_t n) {
  return up256((size_t)n * kBatchAccStride * 8) + up256((size_t)n * 8) + 256;
}

void place_tail(char* base, size_t desc_cap, uint32_t n, unsigned long long*& acc,
                unsigned long long*& out, DevSlot*& slot) {
  acc = (unsigned long long*)(base + desc_cap);
  out = (unsigned long long*)(base + desc_cap + up256((size_t)n * kBatchAccStride * 8));
  slot = (DevSlot*)((char*)out + up256((size_t)n * 8));
}

// Writes the plan's descriptors to `dev` in stream order and fills `a`.
sel_status upload_plan(sel_ctx* ctx, const BatchPlan& bp, char* dev, uint32_t* gtab, BatchArgs& a,
                       const TableBuild** d_builds) {
  std::vector<uint8_t> host(bp.bytes());
  bp.write(host.data(), dev, gtab, a, d_builds);
  return stage_copy(ctx, dev, host.data(), host.size());
}

void release(sel_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ready) (void)hipEventDestroy(b->ready);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  if (b->dev) (void)hipFree(b->dev);
  if (b->h_out) (void)hipHostFree(b->h_out);
  delete b;
}

// Captures the persistent kernel, then the copy of the counts to pinned host
// memory; no memset node (the kernel leaves its accumulators zero).
sel_status capture(sel_batch* b) {
  sel_ctx* ctx = b->ctx;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  hipError_t e;
  const char* where = "";
  do {
    if ((e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) { where = "hipStreamBeginCapture"; break; }
    int le = b->plan.launch(b->args, b->d_builds, b->grid, b->block, b->stream);
    hipError_t ce = hipMemcpyAsync(b->h_out, b->d_out, (size_t)b->n * 8, hipMemcpyDeviceToHost, b->stream);
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (le) { e = (hipError_t)le; where = "batch launch (capture)"; break; }
    if (ce != hipSuccess) { e = ce; where = "hipMemcpyAsync (capture)"; break; }
    if (e != hipSuccess) { where = "hipStreamEndCapture"; break; }
    if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) { where = "hipGraphInstantiate"; break; }
  } while (0);
  if (e != hipSuccess) return hip_err(ctx, e, where);
  return SEL_OK;
}

// Plans, uploads and (re)captures a batch from its current pairs.  The
// graph is captured again only when the launch arguments change; otherwise
// rewriting the descriptors in place refreshes it.
sel_status rebuild(sel_batch* b) {
  sel_ctx* ctx = b->ctx;
  sel_status st = plan_batch(ctx, b->n, b->tabs.data(), b->slot_prog.data(), b->plan);
  if (st != SEL_OK) return st;
  const size_t need = up256(b->plan.bytes());
  const size_t need_gtab = up256(b->plan.gtab_total() * 4);
  if (need > b->desc_cap || need_gtab > b->gtab_cap) {
    if (b->dev) {
      (void)hipStreamSynchronize(b->stream);
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(b->dev);
      b->dev = nullptr;
    }
    const size_t cap = up256(need * 2), gcap = up256(need_gtab * 2);
    const size_t total = cap + tail_bytes(b->n) + gcap;
    HIP_TRY(ctx, hipMalloc(&b->dev, total), "hipMalloc(batch)");
    HIP_TRY(ctx, hipMemsetAsync(b->dev, 0, total, ctx->stream), "hipMemsetAsync(batch)");
    b->desc_cap = cap;
    b->gtab_cap = gcap;
    place_tail((char*)b->dev, cap, b->n, b->d_acc, b->d_out, b->d_slot);
    b->d_gtab = (uint32_t*)((char*)b->dev + cap + tail_bytes(b->n));
  }
  BatchArgs a{};
  const TableBuild* d_builds = nullptr;
  st = upload_plan(ctx, b->plan, (char*)b->dev, b->d_gtab, a, &d_builds);
  if (st != SEL_OK) return st;
  a.acc = b->d_acc;
  a.done = nullptr;
  a.ndone = b->n;
  a.out = b->d_out;
  a.slot = b->d_slot;
  uint32_t grid, block;
  batch_shape(ctx, b->n, b->plan, grid, block);
  const uint32_t lds = b->plan.lds_bytes(block);
  const uint32_t nbuilds = (uint32_t)b->plan.builds.size();
  // the lookup-table launch shapes (one per accumulator width)
  uint32_t lgrid = 0, lblock = 0;
  if (!b->plan.lut.empty())
    for (uint32_t d : {1u, 2u, 4u}) {
      uint32_t g, bl;
      b->plan.lut_shape(d, g, bl);
      lgrid = lgrid * 31u + g;
      lblock = lblock * 31u + bl;
    }
  lblock = lblock * 31u + b->plan.lut_rows;
  const uint32_t llds = b->plan.lut.empty() ? 0u : b->plan.lut.lds_bytes();
  if (b->exec && std::memcmp(&a, &b->args, sizeof a) == 0 && grid == b->grid && block == b->block &&
      lds == b->lds && d_builds == b->d_builds && nbuilds == b->nbuilds &&
      b->plan.table_entries == b->table_entries &&
      std::memcmp(&b->plan.largs, &b->largs, sizeof b->largs) == 0 && lgrid == b->lut_grid &&
      lblock == b->lut_block && llds == b->lut_lds)
    return SEL_OK;
  b->largs = b->plan.largs;
  b->lut_grid = lgrid;
  b->lut_block = lblock;
  b->lut_lds = llds;
  b->args = a;
  b->grid = grid;
  b->block = block;
  b->lds = lds;
  b->d_builds = d_builds;
  b->nbuilds = nbuilds;
  b->table_entries = b->plan.table_entries;
  // the capture stream must see the uploads before its first replay
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  return capture(b);
}

}  // namespace

extern "C" {

sel_status sel_count_batch(sel_ctx* ctx, uint32_t n, const sel_table* const* tables,
                           const sel_program* const* progs, uint64_t* out_counts) {
  if (!ctx || !out_counts) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  BatchPlan bp;
  sel_status st = plan_batch(ctx, n, tables, progs, bp);
  if (st != SEL_OK) return st;
  DeviceGuard g(ctx->device);
  // workspace in the context's batch area: descriptors, then accumulators,
  // counts and the slot
  const size_t desc = up256(bp.bytes());
  const size_t bytes = desc + tail_bytes(n) + up256(bp.gtab_total() * 4);
  if (bytes > ctx->batch_bytes) {
    if (ctx->batch_mem) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(ctx->batch_mem);
      ctx->batch_mem = nullptr;
      ctx->batch_bytes = 0;
    }
    const size_t want = std::max(bytes, size_t(1) << 20);
    HIP_TRY(ctx, hipMalloc(&ctx->batch_mem, want), "hipMalloc(batch)");
    ctx->batch_bytes = want;
  }
  char* base = (char*)ctx->batch_mem;
  BatchArgs a{};
  unsigned long long* acc;
  unsigned long long* outp;
  DevSlot* slot;
  place_tail(base, desc, n, acc, outp, slot);
  // the accumulators move with the descriptor size: clear this call's lines
  int e = sel_launch_fill((uint32_t*)acc, (size_t)n * kBatchAccStride * 2, 0u, ctx->stream);
  if (e) return hip_err(ctx, (hipError_t)e, "accumulator clear");
  const TableBuild* d_builds = nullptr;
  st = upload_plan(ctx, bp, base, (uint32_t*)(base + desc + tail_bytes(n)), a, &d_builds);
  if (st != SEL_OK) return st;
  a.acc = acc;
  a.done = nullptr;
  a.ndone = n;
  a.out = outp;
  a.slot = ctx->slot;
  uint32_t grid, block;
  batch_shape(ctx, n, bp, grid, block);
  {
    TimedLaunch tl(ctx, SEL_K_BATCH);
    e = bp.launch(a, d_builds, grid, block, ctx->stream);
    tl.done();
  }
  if (e) return hip_err(ctx, (hipError_t)e, "batch launch");
  HIP_TRY(ctx, hipMemcpyAsync(ctx->hbatch, a.out, n * 8, hipMemcpyDeviceToHost, ctx->stream),
          "hipMemcpyAsync(batch counts)");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  for (uint32_t i = 0; i < n; ++i) out_counts[i] = ctx->hbatch[i];
  return SEL_OK;
}

sel_status sel_batch_create(sel_ctx* ctx, uint32_t n, const sel_table* const* tables,
                            const sel_program* const* progs, sel_batch** out) {
  if (!ctx || !out) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  *out = nullptr;
  {
    BatchPlan probe;   // validate before allocating anything
    sel_status st = plan_batch(ctx, n, tables, progs, probe);
    if (st != SEL_OK) return st;
  }
  sel_batch* b = new (std::nothrow) sel_batch();
  if (!b) return set_err(ctx, SEL_E_NOMEM, "host allocation failed");
  b->ctx = ctx;
  b->n = n;
  b->tabs.assign(tables, tables + n);
  b->slot_prog.assign(progs, progs + n);
  DeviceGuard g(ctx->device);
  hipError_t e;
  const char* where = "";
  do {
    if ((e = hipHostMalloc((void**)&b->h_out, (size_t)n * 8, hipHostMallocDefault)) != hipSuccess) { where = "hipHostMalloc"; break; }
    if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess) { where = "hipStreamCreate"; break; }
    if ((e = hipEventCreateWithFlags(&b->ready, hipEventDisableTiming)) != hipSuccess) { where = "hipEventCreate"; break; }
  } while (0);
  if (e != hipSuccess) {
    sel_status st = hip_err(ctx, e, where);
    release(b);
    return st;
  }
  sel_status st = rebuild(b);
  if (st != SEL_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    release(b);
    return st;
  }
  *out = b;
  return SEL_OK;
}

sel_status sel_batch_set_program(sel_batch* b, uint32_t i, const sel_program* prog) {
  if (!b) return SEL_E_INVALID;
  sel_ctx* ctx = b->ctx;
  if (!prog || i >= b->n) return set_err(ctx, SEL_E_INVALID, "bad index or NULL program");
  if (prog->table != b->tabs[i])
    return set_err(ctx, SEL_E_INVALID, "program is bound to a different table than the one it replaces");
  DeviceGuard g(ctx->device);
  // a replay still in flight reads the descriptors being replaced
  HIP_TRY(ctx, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  b->slot_prog[i] = prog;
  return rebuild(b);
}

sel_status sel_batch_run(sel_batch* b, uint64_t* out_counts) {
  if (!b || !out_counts) return SEL_E_INVALID;
  sel_ctx* ctx = b->ctx;
  DeviceGuard g(ctx->device);
  // whatever the context's stream enqueued (table uploads, descriptor
  // refreshes) happens before the replay
  HIP_TRY(ctx, hipEventRecord(b->ready, ctx->stream), "hipEventRecord");
  HIP_TRY(ctx, hipStreamWaitEvent(b->stream, b->ready, 0), "hipStreamWaitEvent");
  EventPair ev{};
  const bool timed = ctx->timing;
  if (timed) {
    ev = take_events(ctx);
    HIP_TRY(ctx, hipEventRecord(ev.a, b->stream), "hipEventRecord");
  }
  HIP_TRY(ctx, hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
  if (timed) {
    HIP_TRY(ctx, hipEventRecord(ev.b, b->stream), "hipEventRecord");
    ctx->pending.push_back({SEL_K_BATCH, ev});
  }
  HIP_TRY(ctx, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  for (uint32_t i = 0; i < b->n; ++i) out_counts[i] = b->h_out[i];
  return SEL_OK;
}

void sel_batch_destroy(sel_batch* b) {
  if (!b) return;
  DeviceGuard g(b->ctx->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  release(b);
}

}  // extern "C"

// ---- conjunct counts beside the whole selection's (Ch.1 sec.1.1) ----------

sel_status sel_factor_counts(sel_ctx* ctx, const sel_table* table, const sel_program* prog,
                             uint32_t cap, uint64_t* factor_counts, uint32_t* nfactors,
                             uint64_t* count) {
  if (!ctx) return SEL_E_INVALID;
  if (!nfactors || !count) return set_err(ctx, SEL_E_INVALID, "NULL output");
  if (!table || !prog) return set_err(ctx, SEL_E_INVALID, "NULL handle");
  if (prog->table != table) return set_err(ctx, SEL_E_INVALID, "program is bound to another table");
  const std::vector<DevInstr>& fcode = prog->factor_code.empty() ? prog->host_code : prog->factor_code;
  const auto ranges = and_factors(fcode);
  *nfactors = (uint32_t)ranges.size();
  if (ranges.size() > cap) return set_err(ctx, SEL_E_CAPACITY, "more factors than the output holds");
  if (!factor_counts) return set_err(ctx, SEL_E_INVALID, "factor_counts is NULL");
  // each factor as a program of its own, for the batch planner only (it
  // reads the host copy of the code; the constants stay in prog's device
  // blob)
  std::vector<sel_program> fp(ranges.size());
  std::vector<const sel_program*> progs{prog};
  for (size_t k = 0; k < ranges.size(); ++k) {
    sel_program& f = fp[k];
    f.ctx = ctx;
    f.table = table;
    f.host_code.assign(fcode.begin() + ranges[k].first, fcode.begin() + ranges[k].second);
    f.host_blob = prog->host_blob;
    f.blob_dev = prog->blob_dev;
    f.nins = (uint32_t)f.host_code.size();
    progs.push_back(&f);
  }
  std::vector<const sel_table*> tabs(progs.size(), table);
  std::vector<uint64_t> out(progs.size());
  const sel_status st = sel_count_batch(ctx, (uint32_t)progs.size(), tabs.data(), progs.data(), out.data());
  if (st != SEL_OK) return st;
  *count = out[0];
  for (size_t k = 0; k < ranges.size(); ++k) factor_counts[k] = out[k + 1];
  return SEL_OK;
}

double sel_independence_estimate(uint64_t nrows, uint32_t n, const uint64_t* counts) {
  if (nrows == 0) return 0.0;
  double e = (double)nrows;
  for (uint32_t k = 0; k < n; ++k) e *= (double)counts[k] / (double)nrows;
  return e;
}

