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
  std::vector<const sel_table*> tables;       // distinct, in first-use order
  std::vector<const sel_program*> slot_prog;  // per caller index
  std::vector<uint32_t> slot_to_flat;         // caller index -> BatchProg index
  std::vector<BatchTable> dt;
  std::vector<BatchProg> dp;
  uint64_t total_tiles = 0;
  void* dev = nullptr;                        // tables | progs | acc | out | slot
  BatchTable* d_tables = nullptr;
  BatchProg* d_progs = nullptr;
  unsigned long long* d_acc = nullptr;
  unsigned long long* d_out = nullptr;
  DevSlot* d_slot = nullptr;
  unsigned long long* h_out = nullptr;        // pinned
  hipStream_t stream = nullptr;
  hipEvent_t ready = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t grid = 0, block = 256;
};

namespace {

// Group the (table, program) pairs by table and fill the descriptors.
sel_status plan(sel_ctx* ctx, uint32_t n, const sel_table* const* tables,
                const sel_program* const* progs, sel_batch& b) {
  if (n == 0 || n > (uint32_t)kBatchMaxProgs)
    return set_err(ctx, SEL_E_INVALID, "batch size must be 1..1024");
  if (!tables || !progs) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  b.n = n;
  b.slot_prog.assign(progs, progs + n);
  for (uint32_t i = 0; i < n; ++i) {
    if (!tables[i] || !progs[i]) return set_err(ctx, SEL_E_INVALID, "NULL table or program");
    if (progs[i]->table != tables[i])
      return set_err(ctx, SEL_E_INVALID, "program " + std::to_string(i) + " is bound to another table");
    if (std::find(b.tables.begin(), b.tables.end(), tables[i]) == b.tables.end())
      b.tables.push_back(tables[i]);
  }
  b.slot_to_flat.assign(n, 0);
  b.dt.clear();
  b.dp.clear();
  uint64_t tile = 0;
  for (const sel_table* t : b.tables) {
    BatchTable d{};
    d.nrows = t->nrows;
    d.tile_begin = tile;
    d.row_begin = 0;
    d.prog_begin = (uint32_t)b.dp.size();
    for (uint32_t i = 0; i < n; ++i) {
      if (tables[i] != t) continue;
      b.slot_to_flat[i] = (uint32_t)b.dp.size();
      BatchProg p{};
      p.code = progs[i]->dcode;
      p.nins = progs[i]->nins;
      p.acc_index = (uint32_t)b.dp.size();
      b.dp.push_back(p);
    }
    d.prog_count = (uint32_t)b.dp.size() - d.prog_begin;
    tile += ntiles_of(t->nrows);
    if (ntiles_of(t->nrows) == 0) continue;   // an empty table contributes no tile
    b.dt.push_back(d);
  }
  if (b.dt.empty()) {   // every table empty: keep one zero-row entry
    BatchTable d{};
    b.dt.push_back(d);
  }
  b.total_tiles = tile;
  return SEL_OK;
}

// Launch shape of a batch: fixed by the caller, else tuned for this
// (program count, size) class, else 4 workgroups of 256 per CU.
void batch_shape(sel_ctx* ctx, uint32_t nprogs, uint64_t total_tiles, uint32_t& grid,
                 uint32_t& block) {
  block = 256;
  uint64_t g = 0;
  if (ctx->launch_fixed) {
    block = ctx->launch.block;
    g = ctx->launch.grid;
  } else {
    auto it = ctx->tune.find(tune_key(TK_BATCH, batch_class(nprogs), total_tiles));
    if (it != ctx->tune.end()) {
      block = it->second.block;
      g = it->second.grid;
    }
  }
  if (g == 0) {
    int occ = 1;
    if (sel_batch_occupancy(block, &occ) != 0 || occ < 1) occ = 1;
    g = (uint64_t)std::min(occ, (int)(16 * 64 / block)) * ctx->num_cus;
  }
  const uint64_t need = std::max<uint64_t>(1, (total_tiles + block / 64 - 1) / (block / 64));
  grid = (uint32_t)std::min(g, need);
}

size_t layout(uint32_t n, size_t ntables, size_t& off_progs, size_t& off_acc, size_t& off_out,
              size_t& off_slot) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  off_progs = up(ntables * sizeof(BatchTable));
  off_acc = up(off_progs + n * sizeof(BatchProg));
  off_out = up(off_acc + (size_t)n * kBatchAccStride * 8);
  off_slot = up(off_out + (size_t)n * 8);
  return off_slot + 256;
}

sel_status upload_descriptors(sel_ctx* ctx, sel_batch& b) {
  std::vector<uint8_t> host((char*)b.d_acc - (char*)b.dev);
  std::memcpy(host.data(), b.dt.data(), b.dt.size() * sizeof(BatchTable));
  std::memcpy(host.data() + ((char*)b.d_progs - (char*)b.dev), b.dp.data(), b.dp.size() * sizeof(BatchProg));
  return stage_copy(ctx, b.dev, host.data(), host.size());
}

BatchArgs args_of(const sel_batch& b) {
  BatchArgs a{};
  a.tables = b.d_tables;
  a.progs = b.d_progs;
  a.ntables = (uint32_t)b.dt.size();
  a.nprogs = (uint32_t)b.dp.size();
  a.total_tiles = b.total_tiles;
  a.acc = b.d_acc;
  a.done = nullptr;
  a.ndone = (uint32_t)b.dp.size();
  a.out = b.d_out;
  a.slot = b.d_slot;
  return a;
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

}  // namespace

extern "C" {

sel_status sel_count_batch(sel_ctx* ctx, uint32_t n, const sel_table* const* tables,
                           const sel_program* const* progs, uint64_t* out_counts) {
  if (!ctx || !out_counts) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  sel_batch b;
  sel_status st = plan(ctx, n, tables, progs, b);
  if (st != SEL_OK) return st;
  DeviceGuard g(ctx->device);
  // workspace at the start of the context's batch area: descriptors, then
  // accumulators (zeroed once when the area is created), then counts
  size_t op, oa, oo, os;
  const size_t bytes = layout(n, b.dt.size(), op, oa, oo, os);
  if (bytes > ctx->batch_bytes) {
    if (ctx->batch_mem) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(ctx->batch_mem);
      ctx->batch_mem = nullptr;
      ctx->batch_bytes = 0;
    }
    // accumulators sit at a fixed offset for the largest layout: zero all
    const size_t want = std::max(bytes, size_t(1) << 20);
    HIP_TRY(ctx, hipMalloc(&ctx->batch_mem, want), "hipMalloc(batch)");
    HIP_TRY(ctx, hipMemsetAsync(ctx->batch_mem, 0, want, ctx->stream), "hipMemsetAsync(batch)");
    ctx->batch_bytes = want;
  }
  b.dev = ctx->batch_mem;
  b.d_tables = (BatchTable*)b.dev;
  b.d_progs = (BatchProg*)((char*)b.dev + op);
  b.d_acc = (unsigned long long*)((char*)b.dev + oa);
  b.d_out = (unsigned long long*)((char*)b.dev + oo);
  // the accumulators must be zero: earlier batches left them zero, but a
  // layout with a different table count moves them, so clear this range
  int e = sel_launch_fill((uint32_t*)b.d_acc, (size_t)n * kBatchAccStride * 2, 0u, ctx->stream);
  if (e) return hip_err(ctx, (hipError_t)e, "accumulator clear");
  st = upload_descriptors(ctx, b);
  if (st != SEL_OK) {
    b.dev = nullptr;
    return st;
  }
  BatchArgs a = args_of(b);
  a.slot = ctx->slot;
  uint32_t grid, block;
  batch_shape(ctx, n, b.total_tiles, grid, block);
  {
    TimedLaunch tl(ctx, SEL_K_BATCH);
    e = sel_launch_batch(a, grid, block, ctx->stream);
    tl.done();
  }
  b.dev = nullptr;  // borrowed from the context
  if (e) return hip_err(ctx, (hipError_t)e, "batch launch");
  HIP_TRY(ctx, hipMemcpyAsync(ctx->hbatch, a.out, n * 8, hipMemcpyDeviceToHost, ctx->stream),
          "hipMemcpyAsync(batch counts)");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  for (uint32_t i = 0; i < n; ++i) out_counts[i] = ctx->hbatch[b.slot_to_flat[i]];
  return SEL_OK;
}

sel_status sel_batch_create(sel_ctx* ctx, uint32_t n, const sel_table* const* tables,
                            const sel_program* const* progs, sel_batch** out) {
  if (!ctx || !out) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  *out = nullptr;
  sel_batch* b = new (std::nothrow) sel_batch();
  if (!b) return set_err(ctx, SEL_E_NOMEM, "host allocation failed");
  b->ctx = ctx;
  sel_status st = plan(ctx, n, tables, progs, *b);
  if (st != SEL_OK) {
    delete b;
    return st;
  }
  DeviceGuard g(ctx->device);
  size_t op, oa, oo, os;
  const size_t bytes = layout(n, b->dt.size(), op, oa, oo, os);
  hipError_t e;
  const char* where = "";
  do {
    if ((e = hipMalloc(&b->dev, bytes)) != hipSuccess) { where = "hipMalloc(batch)"; break; }
    if ((e = hipMemset(b->dev, 0, bytes)) != hipSuccess) { where = "hipMemset(batch)"; break; }
    if ((e = hipHostMalloc((void**)&b->h_out, (size_t)n * 8, hipHostMallocDefault)) != hipSuccess) { where = "hipHostMalloc"; break; }
    if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess) { where = "hipStreamCreate"; break; }
    if ((e = hipEventCreateWithFlags(&b->ready, hipEventDisableTiming)) != hipSuccess) { where = "hipEventCreate"; break; }
  } while (0);
  if (e != hipSuccess) {
    st = hip_err(ctx, e, where);
    release(b);
    return st;
  }
  b->d_tables = (BatchTable*)b->dev;
  b->d_progs = (BatchProg*)((char*)b->dev + op);
  b->d_acc = (unsigned long long*)((char*)b->dev + oa);
  b->d_out = (unsigned long long*)((char*)b->dev + oo);
  b->d_slot = (DevSlot*)((char*)b->dev + os);
  st = upload_descriptors(ctx, *b);
  if (st == SEL_OK && hipStreamSynchronize(ctx->stream) != hipSuccess)
    st = set_err(ctx, SEL_E_DEVICE, "hipStreamSynchronize");
  if (st != SEL_OK) {
    release(b);
    return st;
  }
  // capture: the persistent kernel, then the copy of the counts to pinned
  // host memory; no memset node (the kernel leaves its accumulators zero)
  batch_shape(ctx, n, b->total_tiles, b->grid, b->block);
  const BatchArgs a = args_of(*b);
  do {
    if ((e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) { where = "hipStreamBeginCapture"; break; }
    int le = sel_launch_batch(a, b->grid, b->block, b->stream);
    hipError_t ce = hipMemcpyAsync(b->h_out, b->d_out, (size_t)b->dp.size() * 8, hipMemcpyDeviceToHost, b->stream);
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (le) { e = (hipError_t)le; where = "batch launch (capture)"; break; }
    if (ce != hipSuccess) { e = ce; where = "hipMemcpyAsync (capture)"; break; }
    if (e != hipSuccess) { where = "hipStreamEndCapture"; break; }
    if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) { where = "hipGraphInstantiate"; break; }
  } while (0);
  if (e != hipSuccess) {
    st = hip_err(ctx, e, where);
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
  if (prog->table != b->slot_prog[i]->table)
    return set_err(ctx, SEL_E_INVALID, "program is bound to a different table than the one it replaces");
  DeviceGuard g(ctx->device);
  b->slot_prog[i] = prog;
  BatchProg& p = b->dp[b->slot_to_flat[i]];
  p.code = prog->dcode;
  p.nins = prog->nins;
  // the descriptor is device memory the captured kernel reads through a
  // pointer: rewriting it in stream order refreshes the graph without a
  // new capture
  return upload_descriptors(ctx, *b);
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
  for (uint32_t i = 0; i < b->n; ++i) out_counts[i] = b->h_out[b->slot_to_flat[i]];
  return SEL_OK;
}

void sel_batch_destroy(sel_batch* b) {
  if (!b) return;
  DeviceGuard g(b->ctx->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  release(b);
}

}  // extern "C"
