// serve.cpp -- continuous batching of estimate requests (the count queries
// of Ch.3 sec.3.1 and the push-downs of Algorithm 1) over resident tables.
//
// Cooperative scans: every table with pending programs is cut into chunks
// of chunk_rows rows.  A round is ONE batched launch that scans the current
// chunk of every such table for every program attached to it, then advances
// each table to its next chunk (wrapping around).  A program attaches at a
// round boundary and is complete after one revolution over its table (one
// round per chunk); counts of disjoint chunks add up to the exact count.
// Requests arriving while rounds run are admitted as accumulator lines and
// HBM budget free up, and their programs share the next round's scan.
// Push-downs (count, limit check, ascending row ids) run on a second worker
// with its own stream, concurrently with the rounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.h"

using namespace sel;
using namespace selrt;

namespace {

using Clock = std::chrono::steady_clock;

constexpr uint32_t kMaxLines = 4096;        // accumulator lines (programs in flight)
constexpr uint32_t kMaxRoundsInFlight = 4;

struct Request {
  uint64_t ticket = 0;
  Clock::time_point t_submit, t_done;
  std::vector<const sel_table*> tables;
  std::vector<const sel_program*> progs;
  std::vector<uint64_t> counts;
  uint32_t remaining = 0;                   // programs not finished
  bool has_pd = false, pd_done = true;
  const sel_table* pd_table = nullptr;
  const sel_program* pd_prog = nullptr;
  uint64_t pd_max_rows = 0, pd_cap = 0, pd_count = 0;
  uint32_t* pd_out = nullptr;
  sel_status pd_status = SEL_OK;
  uint64_t footprint = 0;
  bool done = false;
  hipEvent_t ready = nullptr;               // the caller's stream at submission
};

struct Active {                             // one attached program
  Request* req;
  uint32_t index;                           // program index in the request
  uint32_t chunks_left;
};

struct Member {                             // an attached program in a round
  Active a;
  uint32_t group;                           // its distinct program's line
  bool last;                                // this round finishes it
};

struct TableState {
  const sel_table* table;
  uint64_t chunk_rows;                      // a multiple of the tile
  uint64_t nchunks;
  uint64_t cur = 0;                         // chunk of the next round
  std::vector<Active> progs;
};

struct RoundSlot {                          // per in-flight round
  void* dev = nullptr;                      // descriptors | out | device tables
  size_t dev_bytes = 0, host_bytes = 0;
  uint8_t* host = nullptr;                  // pinned staging for descriptors
  selrt::BatchPlan plan;                    // this round's descriptors
  unsigned long long* h_out = nullptr;      // pinned, finished counts
  hipEvent_t start_ev = nullptr, done_ev = nullptr;   // the round's device time
  DevSlot* slot = nullptr;                  // ticket of this slot's launches
  std::vector<Member> members;              // programs this round counts for
  uint32_t ngroups = 0;                     // distinct programs (lines) in it
  bool busy = false;
};

}  // namespace

struct sel_server {
  sel_ctx* ctx = nullptr;
  sel_server_config cfg{};
  sel_ctx* pd_ctx = nullptr;                // own stream and scratch for push-downs
  hipStream_t stream = nullptr;             // rounds
  unsigned long long* d_acc = nullptr;      // kMaxLines lines, one per distinct program of a round
  std::vector<RoundSlot> slots;
  std::deque<uint32_t> inflight;            // slot indices, oldest first
  uint32_t next_slot = 0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> incoming;            // submitted, not admitted (FIFO)
  std::deque<Request*> pd_queue;            // admitted push-downs
  std::vector<hipEvent_t> round_waits;      // ready events of newly admitted requests
  std::vector<hipEvent_t> free_events;
  std::unordered_map<uint64_t, Request*> by_ticket;
  std::map<const sel_table*, TableState> tables;
  uint64_t next_ticket = 1;
  uint64_t in_use = 0;                      // admitted footprint
  uint32_t admitted = 0, lines_used = 0;
  bool stop = false;
  std::string error;                        // first device error of a worker

  // statistics
  uint64_t submitted = 0, completed = 0, rejected = 0, rounds = 0, round_programs = 0,
           shared_rounds = 0, round_groups = 0;
  double round_gpu_ms = 0, round_host_ms = 0;
  double round_bytes = 0;                   // algorithmic bytes the rounds read
  uint32_t max_admitted = 0;
  std::vector<double> latencies;
  Clock::time_point t_first{}, t_last{};
  bool any = false;

  std::thread worker, pd_worker;
};

namespace {

// Rows per chunk of a table: 1/rounds_per_cycle of it, capped by chunk_rows,
// whole tiles.
uint64_t chunk_rows_of(const sel_server* s, uint64_t nrows) {
  const uint64_t r = s->cfg.rounds_per_cycle ? s->cfg.rounds_per_cycle : 3;
  uint64_t c = (nrows + r - 1) / r;
  if (s->cfg.chunk_rows) c = std::min<uint64_t>(c, s->cfg.chunk_rows);
  c = std::max<uint64_t>(c, 1);
  return (c + kTileRows - 1) / kTileRows * kTileRows;
}

uint64_t footprint_of(const sel_server* s, const Request& r) {
  uint64_t f = (uint64_t)r.progs.size() * kBatchAccStride * 8;
  for (const sel_program* p : r.progs) f += p->nins * sizeof(DevInstr);
  if (r.has_pd) {
    const uint64_t nt = ntiles_of(r.pd_table->nrows);
    // mask, tile lane maps, tile counts, offsets, ids
    f += nt * kWave * 4 + nt * 8 + 2 * nt * 4 + r.pd_cap * 4;
  }
  return f;
}

// Record the first worker error and wake everyone waiting on the server.
void set_error_locked(sel_server* s, const std::string& msg) {
  if (s->error.empty()) s->error = msg;
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

void finish_request_locked(sel_server* s, Request* r) {
  // every wait on the ready event is enqueued by now: recycle it
  if (r->ready) s->free_events.push_back(r->ready);
  r->ready = nullptr;
  r->done = true;
  r->t_done = Clock::now();
  s->in_use -= r->footprint;
  s->admitted -= 1;
  s->completed += 1;
  s->latencies.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
  s->t_last = r->t_done;
  s->cv_done.notify_all();
  s->cv_work.notify_all();   // budget freed: admission may proceed
}

// Whether the oldest queued request fits the budget and the free lines now.
bool admissible_locked(const sel_server* s) {
  if (s->incoming.empty()) return false;
  const uint64_t budget = s->cfg.hbm_budget_bytes ? s->cfg.hbm_budget_bytes : (1ull << 30);
  const uint32_t max_lines = std::min<uint32_t>(s->cfg.max_programs ? s->cfg.max_programs : kMaxLines, kMaxLines);
  const Request* r = s->incoming.front();
  return s->in_use + r->footprint <= budget && s->lines_used + r->progs.size() <= max_lines;
}

// Admit queued requests in arrival order while budget and lines allow.
void admit_locked(sel_server* s) {
  while (admissible_locked(s)) {
    Request* r = s->incoming.front();
    s->incoming.pop_front();
    s->in_use += r->footprint;
    s->admitted += 1;
    s->max_admitted = std::max(s->max_admitted, s->admitted);
    for (uint32_t i = 0; i < r->progs.size(); ++i) {
      auto it = s->tables.find(r->tables[i]);
      if (it == s->tables.end()) {
        TableState ts;
        ts.table = r->tables[i];
        ts.chunk_rows = chunk_rows_of(s, r->tables[i]->nrows);
        ts.nchunks = std::max<uint64_t>(1, (r->tables[i]->nrows + ts.chunk_rows - 1) / ts.chunk_rows);
        it = s->tables.emplace(r->tables[i], ts).first;
      }
      s->lines_used += 1;
      it->second.progs.push_back(Active{r, i, (uint32_t)it->second.nchunks});
    }
    // the rounds that scan for it start after the caller's earlier work
    if (!r->progs.empty()) s->round_waits.push_back(r->ready);
    if (r->has_pd) {
      s->pd_queue.push_back(r);
      s->cv_work.notify_all();   // wake the push-down worker
    }
    if (r->remaining == 0 && r->pd_done) finish_request_locked(s, r);
  }
}

// Host side of a finished round: add each distinct program's chunk count to
// every request program attached to it (rounds retire in launch order, so a
// program's last round retires after all its earlier ones).
void retire_round(sel_server* s, RoundSlot& rs) {
  float ms = 0;
  if (hipEventElapsedTime(&ms, rs.start_ev, rs.done_ev) != hipSuccess) ms = 0;
  std::lock_guard<std::mutex> lk(s->mu);
  s->round_gpu_ms += ms;
  for (const Member& m : rs.members) {
    m.a.req->counts[m.a.index] += rs.h_out[m.group];
    if (m.last) {
      m.a.req->remaining -= 1;
      s->lines_used -= 1;
      if (m.a.req->remaining == 0 && m.a.req->pd_done) finish_request_locked(s, m.a.req);
    }
  }
  rs.members.clear();
  rs.busy = false;
}

bool wait_oldest(sel_server* s) {
  const uint32_t k = s->inflight.front();
  s->inflight.pop_front();
  if (hipEventSynchronize(s->slots[k].done_ev) != hipSuccess) {
    std::lock_guard<std::mutex> lk(s->mu);
    set_error_locked(s, "round failed on the device");
    return false;
  }
  retire_round(s, s->slots[k]);
  return true;
}

// Bytes per row the programs read together: the element size of every
// column one of them tests, plus 1/8 for every validity bitmap one reads.
// (A table has few columns: the sets are short vectors searched linearly.)
double union_bytes_per_row(const std::vector<const sel_program*>& ps) {
  std::vector<const void*> data, valid;
  auto first_time = [](std::vector<const void*>& seen, const void* x) {
    if (std::find(seen.begin(), seen.end(), x) != seen.end()) return false;
    seen.push_back(x);
    return true;
  };
  double b = 0;
  for (const sel_program* p : ps)
    for (const DevInstr& I : p->host_code) {
      const bool value = I.op == D_RANGE || I.op == D_BITMAP || I.op == D_INLIST;
      if (value && I.data && first_time(data, I.data)) b += type_bytes(I.type);
      if ((value || (I.op >= D_NN_TRUE && I.op <= D_NOTNULL)) && I.valid && first_time(valid, I.valid))
        b += 1.0 / 8.0;
    }
  return b;
}

// Build and launch one round; returns false if there was nothing to do.
// Identical programs (the same compiled program on the same table) attached
// by different requests are evaluated once per chunk; their chunk count is
// handed to each of them.
bool launch_round(sel_server* s) {
  const Clock::time_point t0 = Clock::now();
  RoundSlot& rs = s->slots[s->next_slot];
  BatchPlan& bp = rs.plan;
  bp.clear();
  bp.num_cus = s->ctx->num_cus;
  uint32_t ngroups = 0;
  std::vector<hipEvent_t> waits;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<const sel_program*> gp;
    std::vector<uint32_t> gacc;
    bp.allow_lut = true;   // the lookup-table kernel for the programs it can express
    for (auto& kv : s->tables) {
      TableState& ts = kv.second;
      if (ts.progs.empty()) continue;
      const uint64_t row_begin = ts.cur * ts.chunk_rows;
      const uint64_t row_end = std::min(ts.table->nrows, row_begin + ts.chunk_rows);
      // identical programs of different requests are evaluated once
      std::unordered_map<const sel_program*, uint32_t> group;
      gp.clear();
      gacc.clear();
      const Request* first = nullptr;
      bool shared = false;
      for (Active& a : ts.progs) {
        const sel_program* p = a.req->progs[a.index];
        auto g = group.find(p);
        if (g == group.end()) {
          g = group.emplace(p, ngroups).first;
          gp.push_back(p);
          gacc.push_back(ngroups);
          ++ngroups;
        }
        if (!first) first = a.req;
        else if (a.req != first) shared = true;
        a.chunks_left -= 1;
        rs.members.push_back(Member{a, g->second, a.chunks_left == 0});
      }
      // an empty chunk adds no tile; its programs still finish (count 0)
      bp.add(ts.table, row_begin, row_end, gp.data(), gacc.data(), (uint32_t)gp.size());
      s->round_bytes += (double)(row_end - row_begin) * union_bytes_per_row(gp);
      ts.progs.erase(std::remove_if(ts.progs.begin(), ts.progs.end(),
                                    [](const Active& a) { return a.chunks_left == 0; }),
                     ts.progs.end());
      ts.cur = (ts.cur + 1) % ts.nchunks;
      s->shared_rounds += shared ? 1 : 0;
    }
    // a table with no program attached keeps no state: its chunk geometry
    // is taken afresh from the table when a program next attaches, so a
    // table destroyed and another created at the same address is never
    // scanned with the old one's row count
    for (auto it = s->tables.begin(); it != s->tables.end();) {
      if (it->second.progs.empty()) it = s->tables.erase(it);
      else ++it;
    }
    if (ngroups == 0) {
      rs.members.clear();
      return false;
    }
    rs.ngroups = ngroups;
    s->rounds += 1;
    s->round_groups += ngroups;
    s->round_programs += rs.members.size();
    waits.swap(s->round_waits);
  }
  for (hipEvent_t ev : waits) (void)hipStreamWaitEvent(s->stream, ev, 0);
  // device: descriptors, the counts, the device tables; the descriptors are
  // staged through pinned memory
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o_out = up(bp.bytes());
  const size_t o_gtab = up(o_out + (size_t)ngroups * 8);
  const size_t need_dev = o_gtab + bp.gtab_total() * 4;
  if (need_dev > rs.dev_bytes) {
    if (rs.dev) (void)hipFree(rs.dev);
    rs.dev = nullptr;
    rs.dev_bytes = 0;
    const size_t want = std::max(need_dev * 2, size_t(1) << 16);
    if (hipMalloc(&rs.dev, want) != hipSuccess) {
      std::lock_guard<std::mutex> lk(s->mu);
      set_error_locked(s, "out of memory for round descriptors");
      return false;
    }
    rs.dev_bytes = want;
  }
  if (o_gtab > rs.host_bytes) {
    if (rs.host) (void)hipHostFree(rs.host);
    if (rs.h_out) (void)hipHostFree(rs.h_out);
    rs.host = nullptr;
    rs.h_out = nullptr;
    rs.host_bytes = 0;
    const size_t want = std::max(o_gtab * 2, size_t(1) << 16);
    if (hipHostMalloc((void**)&rs.host, want, 0) != hipSuccess ||
        hipHostMalloc((void**)&rs.h_out, want, 0) != hipSuccess) {
      std::lock_guard<std::mutex> lk(s->mu);
      set_error_locked(s, "out of memory for round descriptors");
      return false;
    }
    rs.host_bytes = want;
  }
  BatchArgs a{};
  const TableBuild* d_builds = nullptr;
  bp.write(rs.host, (char*)rs.dev, (uint32_t*)((char*)rs.dev + o_gtab), a, &d_builds);
  a.acc = s->d_acc;
  a.done = nullptr;                  // every line of the round is read out and reset
  a.ndone = ngroups;
  a.out = (unsigned long long*)((char*)rs.dev + o_out);
  a.slot = rs.slot;
  const uint32_t block = bp.default_block();
  const uint32_t lds = bp.lds_bytes(block);
  int occ = 1;
  if (sel_batch_occupancy(block, lds, &occ) != 0 || occ < 1) occ = 1;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>((uint64_t)std::min(occ, 2) * s->ctx->num_cus, (bp.total_tiles + 7) / 8));
  bool ok = hipEventRecord(rs.start_ev, s->stream) == hipSuccess;
  ok = ok && hipMemcpyAsync(rs.dev, rs.host, o_out, hipMemcpyHostToDevice, s->stream) == hipSuccess;
  ok = ok && bp.launch(a, d_builds, grid, block, s->stream) == 0;
  ok = ok && hipMemcpyAsync(rs.h_out, a.out, (size_t)ngroups * 8, hipMemcpyDeviceToHost, s->stream) == hipSuccess;
  ok = ok && hipEventRecord(rs.done_ev, s->stream) == hipSuccess;
  if (!ok) {
    std::lock_guard<std::mutex> lk(s->mu);
    set_error_locked(s, "round launch failed");
    return false;
  }
  rs.busy = true;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->round_host_ms += std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }
  s->inflight.push_back(s->next_slot);
  s->next_slot = (s->next_slot + 1) % (uint32_t)s->slots.size();
  return true;
}

void worker_main(sel_server* s) {
  (void)hipSetDevice(s->ctx->device);
  const uint32_t depth = std::min<uint32_t>(
      s->cfg.rounds_in_flight ? s->cfg.rounds_in_flight : 1, kMaxRoundsInFlight);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      admit_locked(s);
      bool active = false;
      for (auto& kv : s->tables) active |= !kv.second.progs.empty();
      if (!active && s->inflight.empty()) {
        if (s->stop) break;
        // sleep until a request can be admitted (a finished push-down frees
        // budget and notifies) or the server stops
        s->cv_work.wait(lk, [&] { return s->stop || admissible_locked(s); });
        continue;
      }
    }
    // keep `depth` rounds queued on the device; prepare the next meanwhile
    if (s->inflight.size() >= depth || s->slots[s->next_slot].busy) {
      if (!wait_oldest(s)) break;
      continue;
    }
    if (!launch_round(s)) {
      if (!s->inflight.empty()) {
        if (!wait_oldest(s)) break;
      } else {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->error.empty()) break;
      }
    }
  }
  while (!s->inflight.empty()) {
    if (!wait_oldest(s)) break;
  }
}

void pd_worker_main(sel_server* s) {
  (void)hipSetDevice(s->ctx->device);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->pd_queue.empty(); });
      if (s->pd_queue.empty()) break;   // stop and nothing left
      r = s->pd_queue.front();
      s->pd_queue.pop_front();
    }
    uint64_t cnt = 0;
    (void)hipStreamWaitEvent(s->pd_ctx->stream, r->ready, 0);
    sel_status st = sel_pushdown_rowids(s->pd_ctx, r->pd_table, r->pd_prog, r->pd_max_rows, r->pd_out,
                                        r->pd_cap, &cnt);
    std::lock_guard<std::mutex> lk(s->mu);
    r->pd_status = st;
    r->pd_count = cnt;
    r->pd_done = true;
    if (st == SEL_E_DEVICE || st == SEL_E_NOMEM) set_error_locked(s, sel_last_error(s->pd_ctx));
    if (r->remaining == 0) finish_request_locked(s, r);
  }
}

void release_server(sel_server* s) {
  for (RoundSlot& rs : s->slots) {
    if (rs.done_ev) (void)hipEventDestroy(rs.done_ev);
    if (rs.start_ev) (void)hipEventDestroy(rs.start_ev);
    if (rs.dev) (void)hipFree(rs.dev);
    if (rs.host) (void)hipHostFree(rs.host);
    if (rs.h_out) (void)hipHostFree(rs.h_out);
  }
  if (s->d_acc) (void)hipFree(s->d_acc);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->pd_ctx) sel_ctx_destroy(s->pd_ctx);
  for (auto& kv : s->by_ticket) {
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    delete kv.second;
  }
  for (hipEvent_t ev : s->free_events) (void)hipEventDestroy(ev);
  delete s;
}

}  // namespace

extern "C" {

sel_status sel_server_create(sel_ctx* ctx, const sel_server_config* cfg, sel_server** out) {
  if (!ctx || !out) return set_err(ctx, SEL_E_INVALID, "NULL argument");
  *out = nullptr;
  sel_server* s = new (std::nothrow) sel_server();
  if (!s) return set_err(ctx, SEL_E_NOMEM, "host allocation failed");
  s->ctx = ctx;
  if (cfg) s->cfg = *cfg;
  DeviceGuard g(ctx->device);
  const uint32_t depth = std::min<uint32_t>(s->cfg.rounds_in_flight ? s->cfg.rounds_in_flight : 1, kMaxRoundsInFlight);
  s->slots.resize(depth + 1);
  hipError_t e = hipSuccess;
  const char* where = "";
  do {
    if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess) { where = "hipStreamCreate"; break; }
    const size_t acc_bytes = (size_t)kMaxLines * kBatchAccStride * 8;
    const size_t slot_bytes = 256 * s->slots.size();
    if ((e = hipMalloc((void**)&s->d_acc, acc_bytes + slot_bytes)) != hipSuccess) { where = "hipMalloc(server)"; break; }
    if ((e = hipMemset(s->d_acc, 0, acc_bytes + slot_bytes)) != hipSuccess) { where = "hipMemset(server)"; break; }
    for (size_t k = 0; k < s->slots.size(); ++k) {
      s->slots[k].slot = (DevSlot*)((char*)s->d_acc + acc_bytes + 256 * k);
      if ((e = hipEventCreate(&s->slots[k].done_ev)) != hipSuccess ||
          (e = hipEventCreate(&s->slots[k].start_ev)) != hipSuccess) { where = "hipEventCreate"; break; }
    }
  } while (0);
  if (e != hipSuccess) {
    sel_status st = hip_err(ctx, e, where);
    release_server(s);
    return st;
  }
  sel_status st = sel_ctx_create(ctx->device, SEL_STREAM_OWN, &s->pd_ctx);
  if (st != SEL_OK) {
    set_err(ctx, st, "push-down context");
    release_server(s);
    return st;
  }
  s->worker = std::thread(worker_main, s);
  s->pd_worker = std::thread(pd_worker_main, s);
  *out = s;
  return SEL_OK;
}

sel_status sel_server_submit(sel_server* s, const sel_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return SEL_E_INVALID;
  sel_ctx* ctx = s->ctx;
  if (req->nprog > 0 && (!req->tables || !req->progs)) return set_err(ctx, SEL_E_INVALID, "NULL arrays");
  if (req->nprog == 0 && !req->pd_table) return set_err(ctx, SEL_E_INVALID, "empty request");
  Request* r = new (std::nothrow) Request();
  if (!r) return set_err(ctx, SEL_E_NOMEM, "host allocation failed");
  r->t_submit = Clock::now();
  for (uint32_t i = 0; i < req->nprog; ++i) {
    if (!req->tables[i] || !req->progs[i] || req->progs[i]->table != req->tables[i]) {
      delete r;
      return set_err(ctx, SEL_E_INVALID, "program " + std::to_string(i) + " missing or bound to another table");
    }
    if (batch_slots_alone(req->progs[i]) > kBatchMaxSlots) {
      delete r;
      return set_err(ctx, SEL_E_INVALID, "program " + std::to_string(i) + " has too many leaves to batch");
    }
    r->tables.push_back(req->tables[i]);
    r->progs.push_back(req->progs[i]);
  }
  r->counts.assign(req->nprog, 0);
  r->remaining = req->nprog;
  if (req->pd_table) {
    if (!req->pd_prog || req->pd_prog->table != req->pd_table ||
        (!req->pd_out && req->pd_cap > 0)) {
      delete r;
      return set_err(ctx, SEL_E_INVALID, "bad push-down item");
    }
    r->has_pd = true;
    r->pd_done = false;
    r->pd_table = req->pd_table;
    r->pd_prog = req->pd_prog;
    r->pd_max_rows = req->pd_max_rows;
    r->pd_out = req->pd_out;
    r->pd_cap = req->pd_cap;
  }
  r->footprint = footprint_of(s, *r);
  const uint64_t budget = s->cfg.hbm_budget_bytes ? s->cfg.hbm_budget_bytes : (1ull << 30);
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->error.empty()) {
    delete r;
    return set_err(ctx, SEL_E_DEVICE, s->error);
  }
  if (r->footprint > budget || r->progs.size() > kMaxLines) {
    s->rejected += 1;
    delete r;
    return set_err(ctx, SEL_E_BUSY, "request needs more device memory than the server's budget");
  }
  if (!s->free_events.empty()) {
    r->ready = s->free_events.back();
    s->free_events.pop_back();
  } else if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess) {
    delete r;
    return set_err(ctx, SEL_E_DEVICE, "hipEventCreate");
  }
  {
    DeviceGuard g(ctx->device);
    if (hipEventRecord(r->ready, ctx->stream) != hipSuccess) {
      s->free_events.push_back(r->ready);
      delete r;
      return set_err(ctx, SEL_E_DEVICE, "hipEventRecord");
    }
  }
  r->ticket = s->next_ticket++;
  s->by_ticket[r->ticket] = r;
  s->incoming.push_back(r);
  s->submitted += 1;
  if (!s->any) {
    s->any = true;
    s->t_first = r->t_submit;
  }
  *ticket = r->ticket;
  s->cv_work.notify_all();
  return SEL_OK;
}

sel_status sel_server_poll(sel_server* s, uint64_t ticket, int* done) {
  if (!s || !done) return SEL_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return set_err(s->ctx, SEL_E_INVALID, "unknown ticket");
  *done = it->second->done ? 1 : 0;
  return SEL_OK;
}

sel_status sel_server_wait(sel_server* s, uint64_t ticket, uint64_t* counts, sel_result* res) {
  if (!s) return SEL_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return set_err(s->ctx, SEL_E_INVALID, "unknown ticket");
  Request* r = it->second;
  s->cv_done.wait(lk, [&] { return r->done || !s->error.empty(); });
  if (!r->done) return set_err(s->ctx, SEL_E_DEVICE, s->error);
  if (counts) std::copy(r->counts.begin(), r->counts.end(), counts);
  if (res) {
    res->status = r->pd_status;
    res->pd_count = r->pd_count;
    res->latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  }
  s->by_ticket.erase(it);
  delete r;
  return SEL_OK;
}

sel_status sel_server_get_stats(sel_server* s, sel_server_stats* out, int reset) {
  if (!s || !out) return SEL_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->rejected = s->rejected;
  out->rounds = s->rounds;
  out->round_programs = s->round_programs;
  out->shared_rounds = s->shared_rounds;
  out->max_admitted = s->max_admitted;
  out->round_groups = s->round_groups;
  out->round_gpu_ms = s->round_gpu_ms;
  out->round_host_ms = s->round_host_ms;
  out->round_bytes = s->round_bytes;
  std::vector<double> v = s->latencies;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      size_t k = (size_t)std::min<double>((double)v.size() - 1, std::max(0.0, q * (double)(v.size() - 1) + 0.5));
      return v[k];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_ms = sum / (double)v.size();
    out->max_ms = v.back();
  }
  if (s->any && s->completed) out->elapsed_s = std::chrono::duration<double>(s->t_last - s->t_first).count();
  if (reset) {
    s->submitted = s->completed = s->rejected = s->rounds = s->round_programs = s->shared_rounds = 0;
    s->round_groups = 0;
    s->round_gpu_ms = s->round_host_ms = 0;
    s->round_bytes = 0;
    s->max_admitted = s->admitted;
    s->latencies.clear();
    s->any = false;
  }
  return SEL_OK;
}

void sel_server_destroy(sel_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  if (s->pd_worker.joinable()) s->pd_worker.join();
  DeviceGuard g(s->ctx->device);
  (void)hipStreamSynchronize(s->stream);
  release_server(s);
}

}  // extern "C"
