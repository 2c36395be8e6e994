// Batched and session entry points.
#include <algorithm>
#include <deque>
#include <vector>

#include "vc_internal.h"

namespace vc {
namespace {
inline size_t al(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace
}  // namespace vc

extern "C" {

size_t viecut_batch_workspace_bytes(const viecut_csr *gs, int32_t count, const viecut_params *p) {
  if (!gs || count < 0) return 0;
  size_t tot = 0;
  for (int32_t i = 0; i < count; i++) {
    if (vc::check_args(&gs[i], p)) continue;
    tot += vc::al(vc::work_bytes(gs[i].n, gs[i].nnz));
  }
  return tot + 256;
}

int viecut_mincut_batch(const viecut_csr *gs, int32_t count, const viecut_params *p, void *ws, size_t ws_bytes,
                        void *stream, viecut_result *outs, uint64_t *const *sides) {
  if (!gs || !p || !outs || !sides || count < 0) return VIECUT_EINVAL;
  int first = VIECUT_OK;
  for (int32_t i = 0; i < count; i++) {
    int rc = vc::solve_one(&gs[i], p, nullptr, 0, stream, &outs[i], sides[i], nullptr, nullptr);
    if (rc) {
      outs[i] = viecut_result{};
      outs[i].status_bits = 0x80000000u | (uint32_t)(-rc);
      if (!first) first = rc;
    }
  }
  (void)ws;
  (void)ws_bytes;
  return first;
}

struct viecut_session {
  size_t budget;
  viecut_params p;
  void *stream;
  struct Req { viecut_csr g; uint64_t *side; int64_t id; };
  std::deque<Req> queue;
  std::vector<std::pair<int64_t, viecut_result>> done;
};

int viecut_session_create(size_t hbm_budget, const viecut_params *p, void *stream, viecut_session **out) {
  if (!p || !out) return VIECUT_EINVAL;
  viecut_session *s = new viecut_session();
  s->budget = hbm_budget;
  s->p = *p;
  s->stream = stream;
  *out = s;
  return VIECUT_OK;
}

int viecut_session_submit(viecut_session *s, const viecut_csr *g, uint64_t *side, int64_t request_id) {
  if (!s || !g || !side) return VIECUT_EINVAL;
  int rc = vc::check_args(g, &s->p);
  if (rc) return rc;
  if (vc::work_bytes(g->n, g->nnz) > s->budget) return VIECUT_EBUDGET;
  s->queue.push_back({*g, side, request_id});
  return VIECUT_OK;
}

int viecut_session_step(viecut_session *s, int32_t *n_active) {
  if (!s) return VIECUT_EINVAL;
  if (!s->queue.empty()) {
    viecut_session::Req r = s->queue.front();
    s->queue.pop_front();
    viecut_result res{};
    int rc = vc::solve_one(&r.g, &s->p, nullptr, 0, s->stream, &res, r.side, nullptr, nullptr);
    if (rc) res.status_bits = 0x80000000u | (uint32_t)(-rc);
    s->done.push_back({r.id, res});
  }
  if (n_active) *n_active = (int32_t)s->queue.size();
  return VIECUT_OK;
}

int viecut_session_poll(viecut_session *s, int64_t *ids, viecut_result *outs, int32_t max) {
  if (!s || max < 0) return VIECUT_EINVAL;
  int32_t k = std::min<int32_t>(max, (int32_t)s->done.size());
  for (int32_t i = 0; i < k; i++) {
    if (ids) ids[i] = s->done[i].first;
    if (outs) outs[i] = s->done[i].second;
  }
  s->done.erase(s->done.begin(), s->done.begin() + k);
  return k;
}

void viecut_session_destroy(viecut_session *s) { delete s; }

}  // extern "C"
