// api.cpp -- the C ABI of libsel (include/sel.h): contexts, tables,
// programs, the count query and the push-down calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/sel.h"
#include "sel_device.h"
#include "sel_internal.h"
#include "runtime.h"

using namespace sel;

namespace selrt {

thread_local std::string g_create_error;


sel_status set_err(sel_ctx* ctx, sel_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  else g_create_error = msg;
  return st;
}

sel_status hip_err(sel_ctx* ctx, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return set_err(ctx, e == hipErrorOutOfMemory ? SEL_E_NOMEM : SEL_E_DEVICE, m);
}


uint32_t dev_type(int32_t t) {
  switch (t) {
    case SEL_I8: return T_I8;
    case SEL_I16: return T_I16;
    case SEL_I32: return T_I32;
    case SEL_I64: return T_I64;
    default: return 0;
  }
}

uint32_t type_bytes(uint32_t dt) {
  switch (dt) {
    case T_I8: return 1;
    case T_I16: return 2;
    case T_I32: return 4;
    default: return 8;
  }
}

sel_status ensure_scratch(sel_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->scratch_bytes) return SEL_OK;
  if (ctx->scratch) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
  }
  size_t want = std::max(bytes, size_t(1) << 20);
  HIP_TRY(ctx, hipMalloc(&ctx->scratch, want), "hipMalloc(scratch)");
  ctx->scratch_bytes = want;
  return SEL_OK;
}

EventPair take_events(sel_ctx* ctx) {
  if (!ctx->free_events.empty()) {
    EventPair p = ctx->free_events.back();
    ctx->free_events.pop_back();
    return p;
  }
  EventPair p{};
  (void)hipEventCreate(&p.a);
  (void)hipEventCreate(&p.b);
  return p;
}

TimedLaunch::TimedLaunch(sel_ctx* c, int k, bool timed) : ctx(c), kind(k), on(c->timing && timed) {
  if (on) {
    ev = take_events(ctx);
    (void)hipEventRecord(ev.a, ctx->stream);
  }
}

void TimedLaunch::done() {
  if (on) {
    (void)hipEventRecord(ev.b, ctx->stream);
    ctx->pending.push_back({kind, ev});
    on = false;
  }
}

uint64_t ntiles_of(uint64_t nrows) { return (nrows + kTileRows - 1) / kTileRows; }

uint32_t tune_class_of(double bytes_per_row, uint32_t nins) {
  const uint32_t b = (uint32_t)std::min(63.0, std::floor(bytes_per_row + 0.5));
  const uint32_t l = nins <= 4 ? 0 : nins <= 8 ? 1 : nins <= 16 ? 2 : 3;
  return (b << 2) | l;
}

uint64_t tune_key(int kind, uint32_t cls, uint64_t ntiles) {
  uint32_t lg = 0;
  while ((1ull << lg) < ntiles + 1) ++lg;
  return (uint64_t)kind | ((uint64_t)cls << 4) | ((uint64_t)lg << 24);
}

// Launch configuration of a scan over ntiles wave tiles: fixed if the
// caller set one, else the tuned one of this (kernel, program class, size)
// if the tuner recorded one, else the defaults: 12 resident waves per CU,
// nontemporal loads, one tile per step, every planned bitmap staged (the
// tuner's choices for the 300M-row fact-table scans).
void scan_shape(sel_ctx* ctx, int mode, uint32_t cls, uint64_t ntiles, sel_launch& cfg, uint32_t& grid,
                uint32_t& block) {
  cfg = kDefaultLaunch;
  if (ctx->launch_fixed) {
    cfg = ctx->launch;
  } else {
    auto it = ctx->tune.find(tune_key(mode, cls, ntiles));
    if (it != ctx->tune.end()) cfg = it->second;
  }
  block = cfg.block;
  uint64_t g = cfg.grid;
  if (g == 0) {
    int occ = 0;
    if (block == 256) {
      occ = ctx->occ[mode];
    } else if (sel_scan_occupancy(mode, block, &occ) != 0) {
      occ = 1;
    }
    if (occ < 1) occ = 1;
    const int per_cu = std::min(occ, (int)(kScanWavesPerCu / (block / kWave)));
    g = (uint64_t)per_cu * ctx->num_cus;
  }
  const uint32_t wpb = block / kWave;
  uint64_t need = (ntiles + wpb - 1) / wpb;
  if (need == 0) need = 1;
  grid = (uint32_t)std::min<uint64_t>(need, std::max<uint64_t>(g, 1));
}

bool check_prog(sel_ctx* ctx, const sel_table* t, const sel_program* p) {
  if (!ctx || !t || !p) {
    set_err(ctx, SEL_E_INVALID, "NULL handle");
    return false;
  }
  if (p->table != t) {
    set_err(ctx, SEL_E_INVALID, "program is bound to another table");
    return false;
  }
  return true;
}

sel_status run_scan(sel_ctx* ctx, int mode, uint32_t cls, ScanArgs& a, int kind, bool timed,
                    const std::vector<uint32_t>* stage_end) {
  uint32_t grid, block;
  sel_launch cfg;
  scan_shape(ctx, mode, cls, a.ntiles, cfg, grid, block);
  a.cached = cfg.cached;
  a.tiles_per_step = cfg.tiles_per_step ? cfg.tiles_per_step : 1;
  if (stage_end) limit_stage(a, *stage_end, cfg.stage_words);
  a.slot = ctx->slot;
  TimedLaunch tl(ctx, kind, timed);
  int e = sel_launch_scan(mode, a, grid, block, ctx->stream);
  tl.done();
  if (e != 0) return hip_err(ctx, (hipError_t)e, "scan kernel launch");
  return SEL_OK;
}

// Copy host bytes to device memory in stream order through the pinned
// staging buffer (which is free once the previous such copy has run).
sel_status stage_copy(sel_ctx* ctx, void* dst, const void* src, size_t n) {
  if (n > kStageBytes) return set_err(ctx, SEL_E_INVALID, "staged copy too large");
  HIP_TRY(ctx, hipEventSynchronize(ctx->stage_free), "hipEventSynchronize");
  std::memcpy(ctx->hstage, src, n);
  HIP_TRY(ctx, hipMemcpyAsync(dst, ctx->hstage, n, hipMemcpyHostToDevice, ctx->stream), "hipMemcpyAsync(stage)");
  HIP_TRY(ctx, hipEventRecord(ctx->stage_free, ctx->stream), "hipEventRecord");
  return SEL_OK;
}

sel_status read_out(sel_ctx* ctx, uint64_t* v0, uint64_t* v1) {
  HIP_TRY(ctx, hipMemcpyAsync(ctx->hout, ctx->dout, 2 * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, ctx->stream), "hipMemcpyAsync(count)");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  if (v0) *v0 = ctx->hout[0];
  if (v1) *v1 = ctx->hout[1];
  return SEL_OK;
}

std::vector<ColInfo> col_infos(const sel_column* cols, uint32_t ncols) {
  std::vector<ColInfo> v(ncols);
  for (uint32_t k = 0; k < ncols; ++k) {
    v[k].type = dev_type(cols[k].type);
    v[k].dict_card = cols[k].dict_card;
    v[k].nullable = cols[k].valid != nullptr;
    v[k].data = cols[k].data;
    v[k].valid = cols[k].valid;
  }
  return v;
}

sel_status check_columns(sel_ctx* ctx, uint64_t nrows, uint32_t ncols, const sel_column* cols) {
  if (nrows >= (1ull << 32)) return set_err(ctx, SEL_E_INVALID, "nrows must be < 2^32");
  if (ncols == 0 || ncols > SEL_MAX_COLUMNS || cols == nullptr)
    return set_err(ctx, SEL_E_INVALID, "ncols must be 1..64 with a descriptor array");
  for (uint32_t k = 0; k < ncols; ++k) {
    if (dev_type(cols[k].type) == 0)
      return set_err(ctx, SEL_E_INVALID, "column " + std::to_string(k) + ": unknown type");
    if (nrows > 0 && cols[k].data == nullptr)
      return set_err(ctx, SEL_E_INVALID, "column " + std::to_string(k) + ": NULL data");
    if (((uintptr_t)cols[k].data) % 16 != 0)
      return set_err(ctx, SEL_E_INVALID, "column " + std::to_string(k) + ": data not 16-byte aligned");
    if (((uintptr_t)cols[k].valid) % 4 != 0)
      return set_err(ctx, SEL_E_INVALID, "column " + std::to_string(k) + ": validity not 4-byte aligned");
  }
  return SEL_OK;
}

// The row-id push-down over the workspace at sp (the context's grow-only
// scratch, or the fixed array of the call that allocates nothing).  Every
// word the kernels read there is written earlier in the same call: the mask
// pass writes each tile's count and lane map and the mask words those maps
// name, the tile scan writes every offset and chunk value the compaction
// reads.  So nothing needs clearing between calls.
sel_status pushdown_rowids_with(sel_ctx* ctx, const sel_table* table, const sel_program* prog,
                                uint64_t max_rows, uint32_t* d_out, uint64_t cap,
                                uint64_t* out_count, char* sp, bool timed) {
  const uint64_t ntiles = ntiles_of(table->nrows);
  const RowidScratch L(ntiles);
  const size_t mask_bytes = L.mask, counts_bytes = L.counts, chunk_bytes = L.chunk;
  sel_status st;
  uint32_t* mask = (uint32_t*)sp;
  uint32_t* counts = (uint32_t*)(sp + mask_bytes);
  uint32_t* offsets = (uint32_t*)(sp + mask_bytes + counts_bytes);
  uint32_t* chunk_sums = (uint32_t*)(sp + mask_bytes + 2 * counts_bytes);
  uint32_t* chunk_offs = (uint32_t*)(sp + mask_bytes + 2 * counts_bytes + chunk_bytes);
  uint64_t* lanes = (uint64_t*)(sp + mask_bytes + 2 * counts_bytes + 2 * chunk_bytes);
  ScanArgs a{};
  a.prog = prog->dcode;
  a.nins = prog->nins;
  set_stage(a, prog);
  a.nrows = table->nrows;
  a.ntiles = ntiles;
  a.out = ctx->dout;
  a.mask = mask;
  a.tile_lanes = lanes;
  a.tile_counts = counts;
  st = run_scan(ctx, M_MASK, prog->tune_class, a, SEL_K_MASK, timed, &prog->stage_end);
  if (st != SEL_OK) return st;
  // the scan of tile counts and the compaction are enqueued at once; the
  // compaction reads the published count and writes nothing if it exceeds
  // max_rows or cap, so one wait at the end gives the outcome
  {
    TimedLaunch tl(ctx, SEL_K_SCAN, timed);
    int e = sel_launch_scan_tiles(counts, offsets, chunk_sums, chunk_offs, ntiles, ctx->stream);
    tl.done();
    if (e) return hip_err(ctx, (hipError_t)e, "tile scan launch");
  }
  CompactArgs c{};
  c.mask = mask;
  c.tile_lanes = lanes;
  c.offsets = offsets;
  c.chunk_offs = chunk_offs;
  c.ntiles = ntiles;
  c.out = d_out;
  c.cap = cap;
  c.total = ctx->dout;
  c.limit = std::min(max_rows, cap);
  // one wave per tile: compaction is latency-bound, so every tile gets a
  // wave of its own rather than a grid-stride loop
  const uint32_t block = 256;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((ntiles + 15) / 16, 1u << 20));
  {
    TimedLaunch tl(ctx, SEL_K_COMPACT, timed);
    int e = sel_launch_compact(c, grid, block, ctx->stream);
    tl.done();
    if (e) return hip_err(ctx, (hipError_t)e, "compaction launch");
  }
  uint64_t count = 0;
  st = read_out(ctx, &count, nullptr);   // waits for the compaction too
  if (st != SEL_OK) return st;
  *out_count = count;
  if (count > max_rows) return SEL_OVER_LIMIT;   // Algorithm 1: throw, revert
  if (count > cap) return SEL_E_CAPACITY;
  return SEL_OK;
}

}  // namespace selrt

using namespace selrt;

extern "C" {

// ---------------------------------------------------------------- context --

namespace {
void release_ctx(sel_ctx* ctx) {
  for (auto& p : ctx->pending) ctx->free_events.push_back(p.second);
  for (auto& p : ctx->free_events) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  if (ctx->stage_free) (void)hipEventDestroy(ctx->stage_free);
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  if (ctx->arena_mem) (void)hipFree(ctx->arena_mem);
  if (ctx->batch_mem) (void)hipFree(ctx->batch_mem);
  if (ctx->hbatch) (void)hipHostFree(ctx->hbatch);
  if (ctx->slot) (void)hipFree(ctx->slot);
  if (ctx->hout) (void)hipHostFree(ctx->hout);
  if (ctx->hstage) (void)hipHostFree(ctx->hstage);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}
}  // namespace

sel_status sel_ctx_create(int device, void* hip_stream, sel_ctx** out) {
  if (!out) return set_err(nullptr, SEL_E_INVALID, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return set_err(nullptr, SEL_E_DEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return set_err(nullptr, SEL_E_INVALID, "device index out of range");
  sel_ctx* ctx = new (std::nothrow) sel_ctx();
  if (!ctx) return set_err(nullptr, SEL_E_NOMEM, "host allocation failed");
  ctx->device = device;
  DeviceGuard g(device);
  const char* where = "";
  do {
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) { where = "hipGetDeviceProperties"; break; }
    ctx->num_cus = (uint32_t)prop.multiProcessorCount;
    if (hip_stream != SEL_STREAM_OWN) {
      ctx->stream = (hipStream_t)hip_stream;   // NULL: the null stream
    } else {
      if ((e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking)) != hipSuccess) { where = "hipStreamCreate"; break; }
      ctx->own_stream = true;
    }
    void* dmem = nullptr;
    const size_t dbytes = 256 + 129 * sizeof(DevInstr) + kMaxStage * sizeof(BatchBitmap);
    if ((e = hipMalloc(&dmem, dbytes)) != hipSuccess) { where = "hipMalloc(ctx)"; break; }
    ctx->slot = (DevSlot*)dmem;
    if ((e = hipMemset(dmem, 0, dbytes)) != hipSuccess) { where = "hipMemset(ctx)"; break; }
    ctx->dout = (unsigned long long*)((char*)dmem + 128);
    ctx->dstar = (DevInstr*)((char*)dmem + 256);
    ctx->dtrue = ctx->dstar + 128;
    ctx->dstage = (BatchBitmap*)(ctx->dtrue + 1);
    if ((e = hipMalloc(&ctx->arena_mem, kArenaBytes)) != hipSuccess) { where = "hipMalloc(arena)"; break; }
    ctx->arena.init((char*)ctx->arena_mem, kArenaBytes);
    if ((e = hipHostMalloc((void**)&ctx->hout, 64, hipHostMallocDefault)) != hipSuccess) { where = "hipHostMalloc"; break; }
    if ((e = hipHostMalloc((void**)&ctx->hstage, kStageBytes, hipHostMallocDefault)) != hipSuccess) { where = "hipHostMalloc"; break; }
    if ((e = hipHostMalloc((void**)&ctx->hbatch, kBatchMaxProgs * 8, hipHostMallocDefault)) != hipSuccess) { where = "hipHostMalloc"; break; }
    if ((e = hipEventCreateWithFlags(&ctx->stage_free, hipEventDisableTiming)) != hipSuccess) { where = "hipEventCreate"; break; }
    DevInstr t{};
    t.op = D_TRUE;
    if ((e = hipMemcpy(ctx->dtrue, &t, sizeof t, hipMemcpyHostToDevice)) != hipSuccess) { where = "hipMemcpy(ctx)"; break; }
    // the device address of the fixed workspace, with this device current
    if ((e = (hipError_t)sel_noalloc_scratch(device, &ctx->fixed_scratch)) != hipSuccess) { where = "hipGetSymbolAddress(scratch)"; break; }
  } while (0);
  if (e != hipSuccess) {
    sel_status st = hip_err(nullptr, e, where);
    release_ctx(ctx);
    return st;
  }
  for (int m = 0; m < 3; ++m)
    if (sel_scan_occupancy(m, 256, &ctx->occ[m]) != 0 || ctx->occ[m] < 1) ctx->occ[m] = 1;
  // tuned launch shapes saved earlier (sel_tune_save); a missing or
  // unreadable file is ignored
  if (const char* path = std::getenv("SEL_TUNE_CACHE")) {
    if (sel_tune_load(ctx, path) != SEL_OK) ctx->err.clear();
  }
  *out = ctx;
  return SEL_OK;
}

void sel_ctx_destroy(sel_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  release_ctx(ctx);
}

const char* sel_last_error(const sel_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

uint32_t sel_ctx_num_cus(const sel_ctx* ctx) { return ctx ? ctx->num_cus : 0; }

sel_status sel_ctx_set_launch(sel_ctx* ctx, const sel_launch* launch) {
  if (!ctx) return SEL_E_INVALID;
  if (!launch) {
    ctx->launch = kDefaultLaunch;
    ctx->launch_fixed = false;
    return SEL_OK;
  }
  if (launch->block != 64 && launch->block != 128 && launch->block != 256)
    return set_err(ctx, SEL_E_INVALID, "block must be 64, 128 or 256");
  if (launch->tiles_per_step > 4 || launch->tiles_per_step == 3)
    return set_err(ctx, SEL_E_INVALID, "tiles_per_step must be 0, 1, 2 or 4");
  if (launch->rows_per_lane != 0 && launch->rows_per_lane != 4 && launch->rows_per_lane != 8)
    return set_err(ctx, SEL_E_INVALID, "rows_per_lane must be 0, 4 or 8");
  ctx->launch = *launch;
  ctx->launch_fixed = true;
  return SEL_OK;
}

sel_status sel_ctx_enable_timing(sel_ctx* ctx, int enable) {
  if (!ctx) return SEL_E_INVALID;
  ctx->timing = enable != 0;
  return SEL_OK;
}

sel_status sel_ctx_read_timing(sel_ctx* ctx, sel_timing* out, int reset) {
  if (!ctx || !out) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  DeviceGuard g(ctx->device);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  for (auto& p : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.second.a, p.second.b) == hipSuccess) {
      ctx->ms[p.first] += ms;
      ctx->launches[p.first] += 1;
    }
    ctx->free_events.push_back(p.second);
  }
  ctx->pending.clear();
  for (int k = 0; k < SEL_K_NKINDS; ++k) {
    out->ms[k] = ctx->ms[k];
    out->launches[k] = ctx->launches[k];
    if (reset) {
      ctx->ms[k] = 0.0;
      ctx->launches[k] = 0;
    }
  }
  return SEL_OK;
}

// ----------------------------------------------------------------- tables --

sel_status sel_table_create(sel_ctx* ctx, uint64_t nrows, uint32_t ncols, const sel_column* cols,
                            sel_table** out) {
  if (!ctx || !out) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  *out = nullptr;
  sel_status st = check_columns(ctx, nrows, ncols, cols);
  if (st != SEL_OK) return st;
  sel_table* t = new (std::nothrow) sel_table();
  if (!t) return set_err(ctx, SEL_E_NOMEM, "host allocation failed");
  t->ctx = ctx;
  t->nrows = nrows;
  t->cols.assign(cols, cols + ncols);
  *out = t;
  return SEL_OK;
}

void sel_table_destroy(sel_table* t) { delete t; }

uint64_t sel_table_nrows(const sel_table* t) { return t ? t->nrows : 0; }

// --------------------------------------------------------------- programs --

sel_status sel_program_check(uint64_t nrows, uint32_t ncols, const sel_column* cols,
                             const sel_instr* code, uint32_t n, const void* pool,
                             uint32_t pool_bytes, char* text, size_t text_len, char* err,
                             size_t err_len) {
  std::string e;
  sel_status st = SEL_OK;
  std::string tmp_err;
  if (nrows >= (1ull << 32) || ncols == 0 || ncols > SEL_MAX_COLUMNS || cols == nullptr) {
    st = SEL_E_INVALID;
    e = "invalid table description";
  } else {
    for (uint32_t k = 0; k < ncols; ++k)
      if (dev_type(cols[k].type) == 0) {
        st = SEL_E_INVALID;
        e = "column " + std::to_string(k) + ": unknown type";
      }
  }
  Lowered L;
  if (st == SEL_OK) {
    std::vector<ColInfo> ci = col_infos(cols, ncols);
    st = (sel_status)lower_program(ci.data(), ncols, code, n, (const uint8_t*)pool, pool_bytes, L, e);
  }
  if (err && err_len) std::snprintf(err, err_len, "%s", e.c_str());
  if (text && text_len) std::snprintf(text, text_len, "%s", st == SEL_OK ? L.text.c_str() : "");
  return st;
}

sel_status sel_program_compile(sel_ctx* ctx, const sel_table* table, const sel_instr* code,
                               uint32_t n, const void* pool, uint32_t pool_bytes,
                               sel_program** out) {
  if (!ctx || !table || !out) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  *out = nullptr;
  std::vector<ColInfo> ci = col_infos(table->cols.data(), (uint32_t)table->cols.size());
  Lowered L;
  std::string e;
  int st = lower_program(ci.data(), (uint32_t)ci.size(), code, n, (const uint8_t*)pool, pool_bytes, L, e);
  if (st != SEL_OK) return set_err(ctx, (sel_status)st, e);
  // with range tests merged, the conjuncts as written for factor counts:
  // the same leaves' constants, found in the merged program's blob
  Lowered U;
  bool factors_apart = false;
  if (L.merged) {
    std::string e2;
    if (lower_program(ci.data(), (uint32_t)ci.size(), code, n, (const uint8_t*)pool, pool_bytes, U, e2, false) !=
        SEL_OK)
      return set_err(ctx, SEL_E_INVALID, "unmerged lowering failed: " + e2);
    factors_apart = true;
    for (size_t k = 0; k < U.code.size() && factors_apart; ++k) {
      if (!U.aux_is_offset[k]) continue;
      const DevInstr& u = U.code[k];
      const size_t nb = aux_bytes(u);
      bool found = false;
      for (size_t j = 0; j < L.code.size() && !found; ++j) {
        const DevInstr& l = L.code[j];
        if (!L.aux_is_offset[j] || l.op != u.op || l.data != u.data || l.n != u.n || l.lo != u.lo ||
            l.span != u.span || aux_bytes(l) != nb)
          continue;
        const size_t lo = (size_t)(uintptr_t)l.aux, uo = (size_t)(uintptr_t)u.aux;
        if (lo + nb <= L.blob.size() && uo + nb <= U.blob.size() &&
            std::memcmp(L.blob.data() + lo, U.blob.data() + uo, nb) == 0) {
          U.code[k].aux = l.aux;   // an offset into the merged program's blob
          found = true;
        }
      }
      factors_apart = found;
    }
    if (!factors_apart) return set_err(ctx, SEL_E_INVALID, "unmerged lowering does not match the merged one");
  }
  DeviceGuard g(ctx->device);
  sel_program* p = new (std::nothrow) sel_program();
  if (!p) return set_err(ctx, SEL_E_NOMEM, "host allocation failed");
  p->ctx = ctx;
  p->table = table;
  p->nins = (uint32_t)L.code.size();
  p->depth = L.depth;
  p->text = L.text;
  const size_t code_bytes = L.code.size() * sizeof(DevInstr);
  const size_t blob_bytes = (L.blob.size() + 7) & ~size_t(7);
  // bitmaps a scan stages in LDS (their sources are blob offsets until the
  // blob's device address is known)
  std::vector<BatchBitmap> stage;
  p->stage_words = plan_scan_stage(L.code, stage);
  p->nstage = (uint32_t)stage.size();
  for (const BatchBitmap& b : stage) p->stage_end.push_back(b.lds_word + b.words + 1);
  const size_t total = code_bytes + blob_bytes + stage.size() * sizeof(BatchBitmap);
  p->dev = ctx->arena.alloc(total);
  if (!p->dev) {
    hipError_t he = hipMalloc(&p->dev, total);
    if (he != hipSuccess) {
      delete p;
      return hip_err(ctx, he, "hipMalloc(program)");
    }
    p->own_alloc = true;
  }
  p->dcode = (DevInstr*)p->dev;
  const uintptr_t blob_base = (uintptr_t)p->dev + code_bytes;
  for (size_t k = 0; k < L.code.size(); ++k)
    if (L.aux_is_offset[k]) L.code[k].aux = (const void*)(blob_base + (uintptr_t)L.code[k].aux);
  for (BatchBitmap& b : stage) b.src = (const uint32_t*)(blob_base + (uintptr_t)b.src);
  p->dstage = p->nstage ? (const BatchBitmap*)((char*)p->dev + code_bytes + blob_bytes) : nullptr;
  std::vector<uint8_t> host(total, 0);
  std::memcpy(host.data(), L.code.data(), code_bytes);
  if (!L.blob.empty()) std::memcpy(host.data() + code_bytes, L.blob.data(), L.blob.size());
  if (!stage.empty())
    std::memcpy(host.data() + code_bytes + blob_bytes, stage.data(), stage.size() * sizeof(BatchBitmap));
  sel_status cst = stage_copy(ctx, p->dev, host.data(), total);
  if (cst != SEL_OK) {
    if (p->own_alloc) (void)hipFree(p->dev);
    else ctx->arena.release(p->dev);
    delete p;
    return cst;
  }
  p->host_code = L.code;
  p->host_blob = L.blob;
  p->blob_dev = blob_base;
  if (factors_apart) {
    for (size_t k = 0; k < U.code.size(); ++k)
      if (U.aux_is_offset[k]) U.code[k].aux = (const void*)(blob_base + (uintptr_t)U.code[k].aux);
    p->factor_code = U.code;
  } else {
    p->factor_code = p->host_code;
  }
  double bpr = 0.0;
  for (uint32_t c : L.columns) bpr += type_bytes(ci[c].type);
  bpr += (double)L.valid_columns.size() / 8.0;
  p->bytes_per_row = bpr;
  p->tune_class = tune_class_of(bpr, p->nins);
  *out = p;
  return SEL_OK;
}

void sel_program_destroy(sel_program* p) {
  if (!p) return;
  if (p->dev) {
    DeviceGuard g(p->ctx->device);
    if (p->own_alloc) {
      (void)hipStreamSynchronize(p->ctx->stream);
      (void)hipFree(p->dev);
    } else {
      p->ctx->arena.release(p->dev);  // reused in stream order
    }
  }
  delete p;
}

const char* sel_program_listing(const sel_program* p) { return p ? p->text.c_str() : ""; }

double sel_program_bytes_per_row(const sel_program* p) { return p ? p->bytes_per_row : 0.0; }

// ------------------------------------------------------------------ count --

sel_status sel_count_async(sel_ctx* ctx, const sel_table* table, const sel_program* prog,
                           uint64_t* d_count) {
  if (!check_prog(ctx, table, prog)) return SEL_E_INVALID;
  if (!d_count) return set_err(ctx, SEL_E_INVALID, "d_count is NULL");
  DeviceGuard g(ctx->device);
  ScanArgs a{};
  a.prog = prog->dcode;
  a.nins = prog->nins;
  set_stage(a, prog);
  a.nrows = table->nrows;
  a.ntiles = ntiles_of(table->nrows);
  a.out = (unsigned long long*)d_count;
  return run_scan(ctx, M_COUNT, prog->tune_class, a, SEL_K_COUNT, true, &prog->stage_end);
}

sel_status sel_count(sel_ctx* ctx, const sel_table* table, const sel_program* prog,
                     uint64_t* out_count) {
  if (!out_count) return set_err(ctx, SEL_E_INVALID, "out_count is NULL");
  if (!check_prog(ctx, table, prog)) return SEL_E_INVALID;
  DeviceGuard g(ctx->device);
  ScanArgs a{};
  a.prog = prog->dcode;
  a.nins = prog->nins;
  set_stage(a, prog);
  a.nrows = table->nrows;
  a.ntiles = ntiles_of(table->nrows);
  a.out = ctx->dout;
  sel_status st = run_scan(ctx, M_COUNT, prog->tune_class, a, SEL_K_COUNT, true, &prog->stage_end);
  if (st != SEL_OK) return st;
  return read_out(ctx, out_count, nullptr);
}

// -------------------------------------------------------------- push-down --

uint64_t sel_max_rows(uint64_t nrows, double ratio) {
  if (!(ratio > 0.0)) return 0;   // also NaN
  if (ratio >= 1.0) return nrows;
  // maxSize = R.size * PUSH_DOWN_MAX_SELECTIVITY evaluated in double, as
  // Algorithm 1 states it; for an integer count c, c > maxSize iff
  // c > floor(maxSize)
  const double v = (double)nrows * ratio;
  uint64_t f = (uint64_t)std::floor(v);
  return f > nrows ? nrows : f;
}

sel_status sel_pushdown_rowids(sel_ctx* ctx, const sel_table* table, const sel_program* prog,
                               uint64_t max_rows, uint32_t* d_out, uint64_t cap,
                               uint64_t* out_count) {
  if (!out_count) return set_err(ctx, SEL_E_INVALID, "out_count is NULL");
  if (!check_prog(ctx, table, prog)) return SEL_E_INVALID;
  if (!d_out && cap > 0) return set_err(ctx, SEL_E_INVALID, "d_out is NULL with cap > 0");
  DeviceGuard g(ctx->device);
  sel_status st = ensure_scratch(ctx, RowidScratch(ntiles_of(table->nrows)).total());
  if (st != SEL_OK) return st;
  return pushdown_rowids_with(ctx, table, prog, max_rows, d_out, cap, out_count,
                              (char*)ctx->scratch, true);
}

sel_status sel_pushdown_rowids_noalloc(sel_ctx* ctx, const sel_table* table,
                                       const sel_program* prog, uint64_t max_rows,
                                       uint32_t* d_out, uint64_t cap, uint64_t* out_count) {
  if (!out_count) return set_err(ctx, SEL_E_INVALID, "out_count is NULL");
  if (!check_prog(ctx, table, prog)) return SEL_E_INVALID;
  if (!d_out && cap > 0) return set_err(ctx, SEL_E_INVALID, "d_out is NULL with cap > 0");
  const size_t need = RowidScratch(ntiles_of(table->nrows)).total();
  if (need > kNoAllocScratchBytes)
    return set_err(ctx, SEL_E_INVALID,
                   "table of " + std::to_string(table->nrows) + " rows needs " + std::to_string(need) +
                       " bytes of workspace, more than the fixed " +
                       std::to_string(kNoAllocScratchBytes) + " (use sel_pushdown_rowids)");
  if (!ctx->fixed_scratch) return set_err(ctx, SEL_E_DEVICE, "fixed workspace not set up");
  DeviceGuard g(ctx->device);
  return pushdown_rowids_with(ctx, table, prog, max_rows, d_out, cap, out_count,
                              (char*)ctx->fixed_scratch, false);
}

sel_status sel_pushdown_keybitmap(sel_ctx* ctx, const sel_table* dim, uint32_t key_col,
                                  int64_t key_min, const sel_program* prog, uint32_t* d_bitmap,
                                  uint64_t nbits, uint64_t* out_count) {
  if (!ctx || !dim || !out_count) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  if (prog && prog->table != dim) return set_err(ctx, SEL_E_INVALID, "program is bound to another table");
  if (key_col >= dim->cols.size()) return set_err(ctx, SEL_E_INVALID, "key column out of range");
  const sel_column& kc = dim->cols[key_col];
  if (kc.type != SEL_I32 && kc.type != SEL_I64)
    return set_err(ctx, SEL_E_TYPE, "key column must be int32 or int64");
  if (kc.valid) return set_err(ctx, SEL_E_INVALID, "key column must not have NULLs");
  if (nbits == 0 || nbits > (1ull << 32)) return set_err(ctx, SEL_E_INVALID, "nbits must be 1..2^32");
  if (!d_bitmap) return set_err(ctx, SEL_E_INVALID, "d_bitmap is NULL");
  DeviceGuard g(ctx->device);
  int e = sel_launch_fill(d_bitmap, (nbits + 31) / 32, 0u, ctx->stream);
  if (e) return hip_err(ctx, (hipError_t)e, "bitmap clear");
  ScanArgs a{};
  if (prog) {
    a.prog = prog->dcode;
    a.nins = prog->nins;
    set_stage(a, prog);
  } else {
    a.prog = ctx->dtrue;
    a.nins = 1;
  }
  a.nrows = dim->nrows;
  a.ntiles = ntiles_of(dim->nrows);
  a.out = ctx->dout;
  a.key_data = kc.data;
  a.key_type = dev_type(kc.type);
  a.key_min = key_min;
  a.nbits = nbits;
  a.bitmap = d_bitmap;
  sel_status st = run_scan(ctx, M_KEYBITMAP, prog ? prog->tune_class : 0, a, SEL_K_KEYBITMAP, true,
                           prog ? &prog->stage_end : nullptr);
  if (st != SEL_OK) return st;
  uint64_t count = 0, oor = 0;
  st = read_out(ctx, &count, &oor);
  if (st != SEL_OK) return st;
  *out_count = count;
  if (oor) return set_err(ctx, SEL_E_RANGE, std::to_string(oor) + " qualifying keys outside the bitmap range");
  return SEL_OK;
}

sel_status sel_gather(sel_ctx* ctx, const sel_table* table, const uint32_t* d_ids, uint64_t count,
                      uint32_t ncols, const uint32_t* cols, void* const* d_out,
                      uint32_t* const* d_valid_out) {
  if (!ctx || !table) return set_err(ctx, SEL_E_INVALID, "NULL handle");
  if (table->ctx != ctx) return set_err(ctx, SEL_E_INVALID, "table of another context");
  if (ncols == 0 || ncols > kMaxGatherCols || !cols || !d_out)
    return set_err(ctx, SEL_E_INVALID, "ncols must be 1..16 with column and output arrays");
  if (count >= (1ull << 32)) return set_err(ctx, SEL_E_INVALID, "count must be < 2^32");
  if (count > 0 && !d_ids) return set_err(ctx, SEL_E_INVALID, "d_ids is NULL");
  GatherArgs a{};
  a.ids = d_ids;
  a.count = count;
  a.nrows = table->nrows;
  a.ncols = ncols;
  for (uint32_t c = 0; c < ncols; ++c) {
    if (cols[c] >= table->cols.size()) return set_err(ctx, SEL_E_INVALID, "column index out of range");
    if (count > 0 && !d_out[c]) return set_err(ctx, SEL_E_INVALID, "output column is NULL");
    const sel_column& col = table->cols[cols[c]];
    GatherCol& g = a.cols[c];
    g.src = col.data;
    g.valid = col.valid;
    g.out = d_out[c];
    g.out_valid = d_valid_out ? d_valid_out[c] : nullptr;
    g.width = col.type == SEL_I8 ? 1u : col.type == SEL_I16 ? 2u : col.type == SEL_I32 ? 4u : 8u;
  }
  if (count == 0) return SEL_OK;
  DeviceGuard g(ctx->device);
  a.slot = ctx->slot;
  a.out = ctx->dout;
  const uint32_t block = 256;   // 4 waves, each taking 256 consecutive outputs per step
  const uint64_t want = (count + 4 * block - 1) / (4 * block);
  const uint32_t grid = (uint32_t)std::min<uint64_t>(want, (uint64_t)ctx->num_cus * 8);
  {
    TimedLaunch tl(ctx, SEL_K_GATHER);
    const int e = sel_launch_gather(a, grid, block, ctx->stream);
    tl.done();
    if (e != 0) return hip_err(ctx, (hipError_t)e, "gather kernel launch");
  }
  uint64_t bad = 0;
  const sel_status st = read_out(ctx, nullptr, &bad);
  if (st != SEL_OK) return st;
  if (bad) return set_err(ctx, SEL_E_INVALID, std::to_string(bad) + " row ids >= the table's rows");
  return SEL_OK;
}

}  // extern "C"

namespace {

// The star semi-join as a program over the fact table: one bitmap-probe leaf
// per foreign key (smallest bitmap first; each later probe only looks up rows
// every earlier probe left TRUE or UNKNOWN), ANDed, then AND the optional
// fact predicate.
sel_status build_star_code(sel_ctx* ctx, const sel_table* fact, const sel_program* fact_pred,
                           uint32_t nfk, const uint32_t* fk_cols, const uint32_t* const* d_bitmaps,
                           const uint64_t* nbits, std::vector<DevInstr>& code, double& bpr,
                           int& depth) {
  if (!ctx || !fact || !fk_cols || !d_bitmaps || !nbits)
    return set_err(ctx, SEL_E_INVALID, "NULL argument");
  if (nfk < 1 || nfk > 8) return set_err(ctx, SEL_E_INVALID, "nfk must be 1..8");
  if (fact_pred && fact_pred->table != fact)
    return set_err(ctx, SEL_E_INVALID, "program is bound to another table");
  if (fact_pred && fact_pred->depth + 1 > SEL_MAX_DEPTH)
    return set_err(ctx, SEL_E_INVALID, "fact predicate too deep to combine");
  std::vector<uint32_t> order(nfk);
  for (uint32_t d = 0; d < nfk; ++d) {
    order[d] = d;
    if (fk_cols[d] >= fact->cols.size()) return set_err(ctx, SEL_E_INVALID, "fk column out of range");
    const sel_column& c = fact->cols[fk_cols[d]];
    if (c.type != SEL_I32 && c.type != SEL_I64)
      return set_err(ctx, SEL_E_TYPE, "foreign keys must be int32 or int64");
    if (!d_bitmaps[d]) return set_err(ctx, SEL_E_INVALID, "NULL bitmap");
    if (nbits[d] > (1ull << 32)) return set_err(ctx, SEL_E_INVALID, "nbits must be <= 2^32");
  }
  std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return nbits[x] < nbits[y]; });
  code.clear();
  bpr = fact_pred ? fact_pred->bytes_per_row : 0.0;
  for (uint32_t k = 0; k < nfk; ++k) {
    const uint32_t d = order[k];
    const sel_column& c = fact->cols[fk_cols[d]];
    DevInstr I{};
    if (nbits[d] == 0) {
      I.op = c.valid ? D_NN_FALSE : D_FALSE;
      I.valid = c.valid;
      I.type = dev_type(c.type);
    } else {
      I.op = D_BITMAP;
      I.type = dev_type(c.type);
      I.data = c.data;
      I.valid = c.valid;
      I.lo = 0;
      I.span = nbits[d];
      I.aux = d_bitmaps[d];
      I.flags = k > 0 ? F_GUARD_AND : 0u;
      bpr += type_bytes(I.type);
    }
    if (c.valid) bpr += 1.0 / 8.0;
    code.push_back(I);
    if (k > 0) {
      DevInstr A{};
      A.op = D_AND;
      code.push_back(A);
    }
  }
  depth = nfk > 1 ? 2 : 1;
  if (fact_pred) {
    for (const DevInstr& I : fact_pred->host_code) code.push_back(I);
    DevInstr A{};
    A.op = D_AND;
    code.push_back(A);
    depth = std::max(depth, 1 + fact_pred->depth);
  }
  if (code.size() > 128) return set_err(ctx, SEL_E_INVALID, "combined program too long");
  return SEL_OK;
}

}  // namespace

extern "C" {

sel_status sel_star_count(sel_ctx* ctx, const sel_table* fact, const sel_program* fact_pred,
                          uint32_t nfk, const uint32_t* fk_cols, const uint32_t* const* d_bitmaps,
                          const uint64_t* nbits, uint64_t* out_count) {
  if (!out_count) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  std::vector<DevInstr> code;
  double bpr = 0;
  int depth = 0;
  sel_status st = build_star_code(ctx, fact, fact_pred, nfk, fk_cols, d_bitmaps, nbits, code, bpr, depth);
  if (st != SEL_OK) return st;
  DeviceGuard g(ctx->device);
  st = stage_copy(ctx, ctx->dstar, code.data(), code.size() * sizeof(DevInstr));
  if (st != SEL_OK) return st;
  std::vector<BatchBitmap> stage;
  const uint32_t stage_words = plan_scan_stage(code, stage);
  if (!stage.empty()) {
    st = stage_copy(ctx, ctx->dstage, stage.data(), stage.size() * sizeof(BatchBitmap));
    if (st != SEL_OK) return st;
  }
  ScanArgs a{};
  a.prog = ctx->dstar;
  a.nins = (uint32_t)code.size();
  a.stage = ctx->dstage;
  a.nstage = (uint32_t)stage.size();
  a.stage_words = stage_words;
  a.nrows = fact->nrows;
  a.ntiles = ntiles_of(fact->nrows);
  a.out = ctx->dout;
  std::vector<uint32_t> stage_end;
  for (const BatchBitmap& b : stage) stage_end.push_back(b.lds_word + b.words + 1);
  st = run_scan(ctx, M_COUNT, tune_class_of(bpr, a.nins), a, SEL_K_STAR, true, &stage_end);
  if (st != SEL_OK) return st;
  return read_out(ctx, out_count, nullptr);
}

sel_status sel_program_star(sel_ctx* ctx, const sel_table* fact, const sel_program* fact_pred,
                            uint32_t nfk, const uint32_t* fk_cols, const uint32_t* const* d_bitmaps,
                            const uint64_t* nbits, sel_program** out) {
  if (!out) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  *out = nullptr;
  std::vector<DevInstr> code;
  double bpr = 0;
  int depth = 0;
  sel_status st = build_star_code(ctx, fact, fact_pred, nfk, fk_cols, d_bitmaps, nbits, code, bpr, depth);
  if (st != SEL_OK) return st;
  DeviceGuard g(ctx->device);
  sel_program* p = new (std::nothrow) sel_program();
  if (!p) return set_err(ctx, SEL_E_NOMEM, "host allocation failed");
  p->ctx = ctx;
  p->table = fact;
  p->nins = (uint32_t)code.size();
  p->depth = depth;
  p->bytes_per_row = bpr;
  p->tune_class = tune_class_of(bpr, p->nins);
  p->host_code = code;
  if (fact_pred) {   // the fact predicate's constants, for host-side planning
    p->host_blob = fact_pred->host_blob;
    p->blob_dev = fact_pred->blob_dev;
  }
  p->text = "STAR\n";
  std::vector<BatchBitmap> stage;
  p->stage_words = plan_scan_stage(code, stage);
  p->nstage = (uint32_t)stage.size();
  for (const BatchBitmap& b : stage) p->stage_end.push_back(b.lds_word + b.words + 1);
  const size_t code_bytes = code.size() * sizeof(DevInstr);
  const size_t bytes = code_bytes + stage.size() * sizeof(BatchBitmap);
  p->dev = ctx->arena.alloc(bytes);
  if (!p->dev) {
    hipError_t he = hipMalloc(&p->dev, bytes);
    if (he != hipSuccess) {
      delete p;
      return hip_err(ctx, he, "hipMalloc(program)");
    }
    p->own_alloc = true;
  }
  p->dcode = (DevInstr*)p->dev;
  p->dstage = p->nstage ? (const BatchBitmap*)((char*)p->dev + code_bytes) : nullptr;
  std::vector<uint8_t> image(bytes);
  std::memcpy(image.data(), code.data(), code_bytes);
  if (!stage.empty()) std::memcpy(image.data() + code_bytes, stage.data(), stage.size() * sizeof(BatchBitmap));
  st = stage_copy(ctx, p->dev, image.data(), bytes);
  if (st != SEL_OK) {
    if (p->own_alloc) (void)hipFree(p->dev);
    else ctx->arena.release(p->dev);
    delete p;
    return st;
  }
  *out = p;
  return SEL_OK;
}

}  // extern "C"
