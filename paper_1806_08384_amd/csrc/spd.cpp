// spd.cpp -- the push-down decision of Algorithm 1 (Ch.4 sec.4.2,
// "Selective Selection Push-Down") over the exact-count path: a size-ordered
// queue of a query's relations above PUSH_DOWN_MIN_TABLE_SIZE, the largest
// one left for the probe, and for each other relation Execute(compound,
// true, maxSize): its exact count, compared with maxSize = R.size *
// PUSH_DOWN_MAX_SELECTIVITY, then either the materialised sigma(R) or a
// reverted push-down.  Host logic only; every count and every id list comes
// from sel_pushdown_rowids.
#include <algorithm>
#include <cmath>
#include <vector>

#include "runtime.h"

using selrt::set_err;

sel_status sel_select_pushdown(sel_ctx* ctx, uint32_t n, const sel_spd_relation* rels,
                               uint64_t min_table_size, double max_selectivity,
                               sel_spd_result* out) {
  if (!ctx) return SEL_E_INVALID;
  if (n == 0 || !rels || !out) return set_err(ctx, SEL_E_INVALID, "no relations or no result array");
  if (std::isnan(max_selectivity)) return set_err(ctx, SEL_E_INVALID, "max_selectivity is NaN");
  for (uint32_t i = 0; i < n; ++i) {
    const sel_spd_relation& r = rels[i];
    if (!r.table || r.table->ctx != ctx) return set_err(ctx, SEL_E_INVALID, "NULL or foreign table");
    if (r.pred && r.pred->table != r.table)
      return set_err(ctx, SEL_E_INVALID, "selection bound to another table");
    if (r.pred && !r.d_out && r.cap > 0) return set_err(ctx, SEL_E_INVALID, "d_out is NULL with cap > 0");
  }
  // the queue: relations above the size threshold, largest first; equal
  // sizes keep their input order
  std::vector<uint32_t> queue;
  for (uint32_t i = 0; i < n; ++i) {
    sel_spd_result& o = out[i];
    o = sel_spd_result{};
    o.order = UINT32_MAX;
    o.max_rows = sel_max_rows(rels[i].table->nrows, max_selectivity);
    if (rels[i].table->nrows > min_table_size) queue.push_back(i);
    else o.decision = SEL_SPD_SMALL;
  }
  std::stable_sort(queue.begin(), queue.end(), [&](uint32_t a, uint32_t b) {
    return rels[a].table->nrows > rels[b].table->nrows;
  });
  if (queue.empty()) return SEL_OK;
  // the largest relation is the one to be probed: no push-down on it
  out[queue.front()].decision = SEL_SPD_PROBE;
  for (size_t k = 1; k < queue.size(); ++k) {
    const uint32_t i = queue[k];
    const sel_spd_relation& r = rels[i];
    sel_spd_result& o = out[i];
    o.order = (uint32_t)(k - 1);
    if (!r.pred) {
      o.decision = SEL_SPD_NO_PRED;
      continue;
    }
    uint64_t cnt = 0;
    const sel_status st = sel_pushdown_rowids(ctx, r.table, r.pred, o.max_rows, r.d_out, r.cap, &cnt);
    if (st < 0) return st;
    o.status = st;
    o.count = cnt;
    o.decision = st == SEL_OK ? SEL_SPD_PUSHED : SEL_SPD_REVERTED;
  }
  return SEL_OK;
}
