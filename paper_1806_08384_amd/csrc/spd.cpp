// spd.cpp -- the push-down decision of Algorithm 1 (Ch.4 sec.4.2,
// "Selective Selection Push-Down") over the exact-count path: a size-ordered
// queue of a query's relations above PUSH_DOWN_MIN_TABLE_SIZE, the largest
// one left for the probe, and for each other relation Execute(compound,
// true, maxSize): its exact count, compared with maxSize = R.size *
// PUSH_DOWN_MAX_SELECTIVITY, then either the materialised sigma(R) or a
// reverted push-down.  Host logic only; every count and every id list comes
// from sel_pushdown_rowids.  Also the join-size formula of Ch.1 sec.1.1
// that those exact counts feed, for ordering a star query's joins.
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

// ---- join sizes from exact selection counts (Ch.1 sec.1.1) ---------------

double sel_join_size(double r_rows, double s_rows, double v_r, double v_s) {
  const double v = std::max(v_r, v_s);
  return v > 0.0 ? r_rows * s_rows / v : 0.0;
}

double sel_star_plan_cost(double fact_rows, uint32_t ndims, const double* dim_rows,
                          const double* sel_rows, const uint32_t* order, double* inter) {
  if (ndims == 0 || ndims > 64 || !dim_rows || !sel_rows || !order) return -1.0;
  uint64_t seen = 0;
  for (uint32_t k = 0; k < ndims; ++k) {
    if (order[k] >= ndims || (seen >> order[k]) & 1u) return -1.0;
    seen |= 1ull << order[k];
  }
  // the intermediate keeps one row per fact row whose key survives: the
  // fact side holds dim_rows[d] distinct keys, the selected dimension
  // sel_rows[d] of them
  double cur = fact_rows, total = 0.0;
  for (uint32_t k = 0; k < ndims; ++k) {
    const uint32_t d = order[k];
    cur = sel_join_size(cur, sel_rows[d], dim_rows[d], sel_rows[d]);
    if (inter) inter[k] = cur;
    total += cur;
  }
  return total;
}

sel_status sel_star_plan_order(double fact_rows, uint32_t ndims, const double* dim_rows,
                               const double* sel_rows, uint32_t* order, double* cost) {
  if (ndims == 0 || ndims > 64 || !dim_rows || !sel_rows || !order) return SEL_E_INVALID;
  for (uint32_t d = 0; d < ndims; ++d)
    if (!(dim_rows[d] > 0.0) || !(sel_rows[d] >= 0.0) || sel_rows[d] > dim_rows[d]) return SEL_E_INVALID;
  // each join multiplies the running size by the dimension's retained
  // fraction, so the sum of the running sizes is least when the smallest
  // fractions come first
  for (uint32_t d = 0; d < ndims; ++d) order[d] = d;
  std::stable_sort(order, order + ndims, [&](uint32_t a, uint32_t b) {
    return sel_rows[a] / dim_rows[a] < sel_rows[b] / dim_rows[b];
  });
  if (cost) *cost = sel_star_plan_cost(fact_rows, ndims, dim_rows, sel_rows, order, nullptr);
  return SEL_OK;
}

