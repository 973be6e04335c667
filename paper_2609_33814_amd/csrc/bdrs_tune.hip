// Tile-shape autotuner behind bdrs_autotune / bdrs_tune_* (include/bdrs.h).
//
// The tunable of a sweep launch is its number of input splits: a work item is
// a block of kSweepBlock outputs against ceil(ntiles_in / splits) input tiles.
// More splits give more work items (better fill of the 256 CUs on small
// problems) at the price of more partial records to write and merge.  The
// tuner times candidate counts on the caller's problem and keeps the fastest
// per direction in a table keyed by the exact shape (dim, m, n) that
// make_layout consults.
#include "bdrs_host.h"

#include <algorithm>
#include <mutex>
#include <vector>

using namespace bdrs;

namespace bdrs_host {
namespace {

std::mutex g_tune_mu;
std::vector<bdrs_tune_entry> g_tune;

constexpr size_t kMaxPartialBytes = size_t(1) << 30;  // per candidate, both directions

// Powers of two from h/16 to 16h around the heuristic's count h, each
// normalised, plus h itself; candidates whose partial records would exceed
// kMaxPartialBytes are dropped (h is always kept).
std::vector<int> split_candidates(int np_out, int ntiles_in) {
  const int h = choose_splits(np_out, ntiles_in);
  std::vector<int> c{h};
  for (long long s = 1; s <= ntiles_in && s <= 16LL * h; s *= 2) {
    if (16 * s < h) continue;
    const int v = normalize_splits((int)s, ntiles_in);
    if ((size_t)v * (size_t)np_out * kPartialSlot <= kMaxPartialBytes) c.push_back(v);
  }
  std::sort(c.begin(), c.end());
  c.erase(std::unique(c.begin(), c.end()), c.end());
  return c;
}

double median_of(std::vector<float> v) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const size_t h = v.size() / 2;
  return v.size() % 2 ? (double)v[h] : 0.5 * ((double)v[h - 1] + (double)v[h]);
}

int tiles_of(int count) { return (count + kTile - 1) / kTile; }

}  // namespace

bool tuned_splits(int dim, int m, int n, int* splits_row, int* splits_col) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const bdrs_tune_entry& e : g_tune) {
    if (e.dim == dim && e.m == m && e.n == n) {
      *splits_row = e.splits_row;
      *splits_col = e.splits_col;
      return true;
    }
  }
  return false;
}

}  // namespace bdrs_host

using namespace bdrs_host;

extern "C" {

bdrs_status bdrs_tune_set(const bdrs_tune_entry* e) {
  if (!e) return fail(BDRS_E_INVALID, "entry is NULL");
  if (e->dim < 1 || e->dim > 3) return fail(BDRS_E_INVALID, "dim must be 1, 2 or 3: %d", e->dim);
  if (e->m < 1 || e->m > (1 << 30) || e->n < 1 || e->n > (1 << 30))
    return fail(BDRS_E_INVALID, "m and n must lie in [1, 2^30]");
  if (e->splits_row < 1 || e->splits_col < 1) return fail(BDRS_E_INVALID, "split counts must be >= 1");
  bdrs_tune_entry v = *e;
  v.splits_row = normalize_splits(v.splits_row, tiles_of(v.n));
  v.splits_col = normalize_splits(v.splits_col, tiles_of(v.m));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (bdrs_tune_entry& x : g_tune) {
    if (x.dim == v.dim && x.m == v.m && x.n == v.n) {
      x = v;
      return BDRS_OK;
    }
  }
  g_tune.push_back(v);
  return BDRS_OK;
}

bdrs_status bdrs_tune_get(int32_t index, bdrs_tune_entry* out, int32_t* count) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (count) *count = (int32_t)g_tune.size();
  if (!out) return BDRS_OK;
  if (index < 0 || (size_t)index >= g_tune.size())
    return fail(BDRS_E_INVALID, "tune table index %d out of range (%zu entries)", index, g_tune.size());
  *out = g_tune[index];
  return BDRS_OK;
}

bdrs_status bdrs_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return BDRS_OK;
}

bdrs_status bdrs_autotune_workspace_size(const bdrs_params* p, size_t* bytes) {
  bdrs_status st = check_sizes(p);
  if (st != BDRS_OK) return st;
  if (!bytes) return fail(BDRS_E_INVALID, "bytes is NULL");
  const Layout L0 = make_layout(p->m, p->n, p->dim);
  const std::vector<int> cr = split_candidates(L0.R.np, L0.C.ntiles);
  const std::vector<int> cc = split_candidates(L0.C.np, L0.R.ntiles);
  *bytes = make_layout(p->m, p->n, p->dim, cr.back(), cc.back()).total;
  return BDRS_OK;
}

bdrs_status bdrs_autotune(const bdrs_params* p, int32_t rounds, bdrs_tune_entry* out) {
  if (!out) return fail(BDRS_E_INVALID, "out is NULL");
  bdrs_status st = check_sizes(p);
  if (st != BDRS_OK) return st;
  if (rounds < 1 || rounds > 1000) return fail(BDRS_E_INVALID, "rounds must lie in [1, 1000]: %d", rounds);
  const Layout L0 = make_layout(p->m, p->n, p->dim);
  const std::vector<int> cr = split_candidates(L0.R.np, L0.C.ntiles);
  const std::vector<int> cc = split_candidates(L0.C.np, L0.R.ntiles);
  const size_t need = make_layout(p->m, p->n, p->dim, cr.back(), cc.back()).total;
  if ((st = check_params(p, need)) != BDRS_OK) return st;
  if ((st = check_device()) != BDRS_OK) return st;

  std::vector<float> hx, hy;
  std::vector<double> hr, hc;
  if ((st = download_inputs(p, hx, hy, hr, hc)) != BDRS_OK) return st;
  bdrs_solver s = nullptr;
  st = create_from_host(p, hx.data(), hy.data(), hr.data(), hc.data(), &s, cr.back(), cc.back());
  if (st != BDRS_OK) return st;

  const int nr = (int)cr.size(), nc = (int)cc.size(), K = std::max(nr, nc);
  const int hr_split = choose_splits(L0.R.np, L0.C.ntiles), hc_split = choose_splits(L0.C.np, L0.R.ntiles);
  std::vector<std::vector<float>> tr(nr), tc(nc);
  std::vector<hipEvent_t> ev(3 * (size_t)K, nullptr);
  hipError_t e = hipSuccess;
  for (auto& x : ev)
    if (e == hipSuccess) e = hipEventCreate(&x);
  // warm-up into the regime where a solve spends most of its sweeps (at low
  // temperature most input tiles are skipped): up to 500 iterations, at most
  // about 2e13 implicit entries, at least 10
  const double per_iter = 2.0 * (double)p->m * (double)p->n;
  const int warm = (int)std::max(10.0, std::min(500.0, std::floor(2e13 / per_iter)));
  if (e == hipSuccess && (st = bdrs_step(s, warm)) != BDRS_OK) e = hipErrorUnknown;
  LaunchCtx& c = s->ctx;
  for (int r = 0; r < rounds && e == hipSuccess; ++r) {
    for (int i = 0; i < K && e == hipSuccess; ++i) {
      const int sr = cr[i % nr], sc = cc[i % nc];
      c.splits_row = sr;
      c.splits_col = sc;
      e = hipEventRecord(ev[3 * i], c.stream);
      if (e == hipSuccess) e = launch_sweep(c, false, false, sr, -1.0, 0);
      if (e == hipSuccess) e = launch_finish(c, false, kFinishRow, sr, -1.0, nullptr, 0);
      if (e == hipSuccess) e = hipEventRecord(ev[3 * i + 1], c.stream);
      if (e == hipSuccess) e = launch_sweep(c, true, false, sc, -1.0, 0);
      if (e == hipSuccess) e = launch_finish(c, true, kFinishCol, sc, -1.0, nullptr, 0);
      if (e == hipSuccess) e = hipEventRecord(ev[3 * i + 2], c.stream);
      if (e == hipSuccess) e = launch_advance(c.ctrl, 1, c.stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    for (int i = 0; i < K && e == hipSuccess; ++i) {
      float a = 0.f, b = 0.f;
      e = hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]);
      if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[3 * i + 1], ev[3 * i + 2]);
      // every candidate gets the same number of samples per round
      if (e == hipSuccess && i < nr) tr[i].push_back(a * 1e3f);
      if (e == hipSuccess && i < nc) tc[i].push_back(b * 1e3f);
    }
  }
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  bdrs_destroy(s);
  if (st != BDRS_OK) return st;
  if (e != hipSuccess) return hip_status(e, "autotune");

  bdrs_tune_entry best{};
  best.dim = p->dim;
  best.m = p->m;
  best.n = p->n;
  best.candidates = K;
  best.us_row = best.us_col = 1e300;
  for (int i = 0; i < nr; ++i) {
    const double t = median_of(tr[i]);
    if (t < best.us_row) best.us_row = t, best.splits_row = cr[i];
    if (cr[i] == hr_split) best.us_row_default = t;
  }
  for (int i = 0; i < nc; ++i) {
    const double t = median_of(tc[i]);
    if (t < best.us_col) best.us_col = t, best.splits_col = cc[i];
    if (cc[i] == hc_split) best.us_col_default = t;
  }
  if ((st = bdrs_tune_set(&best)) != BDRS_OK) return st;
  *out = best;
  return BDRS_OK;
}

}  // extern "C"
