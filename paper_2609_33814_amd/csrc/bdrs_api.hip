// Host runtime behind the C ABI of include/bdrs.h.
//
// Responsibilities: argument checks (host only, before any HIP call), the
// layout of the caller's device workspace, the tile order of the points
// (Morton order, so that each 64-point tile is spatially compact), and the
// iteration / certificate loop of Algorithm 1 with the best-bound stopping
// rule.
#include "bdrs_host.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

using namespace bdrs;

namespace bdrs_host {

thread_local std::string g_err;

bdrs_status fail(bdrs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(BDRS_E_DEVICE, "HIP error %s in %s", hipGetErrorString(e_), #expr);     \
  } while (0)



SideShape side_shape(int count) {
  SideShape s;
  s.count = count;
  s.ntiles = (count + kTile - 1) / kTile;
  s.np = (s.ntiles * kTile + kPad - 1) / kPad * kPad;
  return s;
}


int normalize_splits(int s, int ntiles_in) {
  s = std::max(1, std::min(s, ntiles_in));
  const int tps = (ntiles_in + s - 1) / s;
  return (ntiles_in + tps - 1) / tps;
}

Layout make_layout(int m, int n, int dim, int reserve_row, int reserve_col, bool keep_best) {
  Layout L{};
  L.keep_best = keep_best;
  L.R = side_shape(m);
  L.C = side_shape(n);
  L.splits_row = choose_splits(L.R.np, L.C.ntiles);
  L.splits_col = choose_splits(L.C.np, L.R.ntiles);
  int sr = 0, sc = 0;
  if (tuned_splits(dim, m, n, &sr, &sc)) {
    L.splits_row = normalize_splits(sr, L.C.ntiles);
    L.splits_col = normalize_splits(sc, L.R.ntiles);
  }
  L.splits_max = std::max(L.splits_row, L.splits_col);
  const int npmax = std::max(L.R.np, L.C.np);
  L.cert_blocks = std::max(1, std::min(256, npmax / kBlock));
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.ctrl = take(sizeof(Ctrl));
  auto side = [&](const SideShape& s, size_t& abs, size_t& off, size_t& tile, size_t& geom, size_t& A,
                  size_t& perm, size_t& marg, size_t& logm, size_t& iperm, size_t& hint) {
    abs = take(sizeof(float) * (size_t)dim * s.np);
    off = take(sizeof(float) * (size_t)s.ntiles * dim * kTile);
    tile = take(sizeof(TileRec) * (size_t)s.ntiles);
    geom = take(sizeof(TileGeom) * (size_t)s.ntiles);
    A = take(sizeof(float) * (size_t)s.np);
    perm = take(sizeof(int) * (size_t)s.np);
    marg = take(sizeof(double) * (size_t)s.np);
    logm = take(sizeof(double) * (size_t)s.np);
    iperm = take(sizeof(int) * (size_t)s.count);
    hint = take(sizeof(int) * (size_t)s.np);
  };
  side(L.R, L.r_abs, L.r_off, L.r_tile, L.r_geom, L.r_A, L.r_perm, L.r_marg, L.r_logm, L.r_iperm, L.r_hint);
  side(L.C, L.c_abs, L.c_off, L.c_tile, L.c_geom, L.c_A, L.c_perm, L.c_marg, L.c_logm, L.c_iperm, L.c_hint);
  L.la = take(sizeof(double) * L.R.np);
  L.lah = take(sizeof(double) * L.R.np);
  L.lb1 = take(sizeof(double) * L.C.np);
  L.lb2 = take(sizeof(double) * L.C.np);
  L.lbh = take(sizeof(double) * L.C.np);
  L.lt0 = take(sizeof(double) * L.C.np);
  L.lt1 = take(sizeof(double) * L.C.np);
  L.mu = take(sizeof(double) * L.C.np);
  L.logs = take(sizeof(double) * L.C.np);
  L.pvec = take(sizeof(double) * L.R.np);
  L.cert_part = take(sizeof(double) * 2 * (size_t)L.cert_blocks * 8);
  L.cert_out = take(sizeof(double) * kCertSlots);
  L.plan_row = take(sizeof(double) * L.R.np);
  L.plan_col = take(sizeof(double) * L.C.np);
  L.plan_aux = take(sizeof(double) * L.R.np);
  L.plan_stats = take(sizeof(double) * kCertSlots);
  L.tile_total = take(sizeof(unsigned long long));
  L.part_ref = take(sizeof(double) * (size_t)npmax);
  if (keep_best) {
    L.best_la = take(sizeof(double) * L.R.np);
    L.best_lah = take(sizeof(double) * L.R.np);
    L.best_lb1 = take(sizeof(double) * L.C.np);
    L.best_lb2 = take(sizeof(double) * L.C.np);
    L.best_lbh = take(sizeof(double) * L.C.np);
    L.best_lt0 = take(sizeof(double) * L.C.np);
    L.best_lt1 = take(sizeof(double) * L.C.np);
    L.best_hr = take(sizeof(int) * L.R.np);
    L.best_hc = take(sizeof(int) * L.C.np);
  }
  // partial records last: every other offset is independent of the split counts
  const size_t rows_rec = (size_t)std::max(L.splits_row, reserve_row) * L.R.np;
  const size_t cols_rec = (size_t)std::max(L.splits_col, reserve_col) * L.C.np;
  L.part = take((size_t)kPartialSlot * std::max(rows_rec, cols_rec));
  // one evaluated-tile count per (split, output wavefront) of a sweep (profiling)
  L.tile_count = take(sizeof(unsigned) * (std::max(rows_rec, cols_rec) / kTile));
  L.total = o;
  return L;
}

bdrs_status check_sizes(const bdrs_params* p) {
  if (!p) return fail(BDRS_E_INVALID, "params is NULL");
  if (p->m < 1 || p->m > (1 << 30)) return fail(BDRS_E_INVALID, "m out of range [1, 2^30]: %d", p->m);
  if (p->n < 1 || p->n > (1 << 30)) return fail(BDRS_E_INVALID, "n out of range [1, 2^30]: %d", p->n);
  if (p->dim < 1 || p->dim > 3) return fail(BDRS_E_INVALID, "dim must be 1, 2 or 3: %d", p->dim);
  return BDRS_OK;
}

bdrs_status check_params(const bdrs_params* p, size_t need) {
  bdrs_status st = check_sizes(p);
  if (st != BDRS_OK) return st;
  if (!p->x) return fail(BDRS_E_INVALID, "x is NULL");
  if (!p->y) return fail(BDRS_E_INVALID, "y is NULL");
  if (!p->r) return fail(BDRS_E_INVALID, "r is NULL");
  if (!p->c) return fail(BDRS_E_INVALID, "c is NULL");
  if (!(std::isfinite(p->cost_scale) && p->cost_scale > 0))
    return fail(BDRS_E_INVALID, "cost_scale must be finite and > 0");
  if (!(std::isfinite(p->eta) && p->eta > 0)) return fail(BDRS_E_INVALID, "eta must be finite and > 0");
  if (!(p->lambda >= 1.0 && p->lambda < 2.0)) return fail(BDRS_E_INVALID, "lambda must lie in [1, 2)");
  if (!(std::isfinite(p->omega) && p->omega > 0))
    return fail(BDRS_E_INVALID, "omega must be finite and > 0 (a bound Omega >= osc(C), Prop. 3)");
  const uint32_t known = BDRS_F_REPAIR | BDRS_F_OLD_KERNEL | BDRS_F_NO_MOMENTUM | BDRS_F_DEBIASED | BDRS_F_NO_GRAPH |
                         BDRS_F_KEEP_BEST_STATE;
  if (p->flags & ~known) return fail(BDRS_E_INVALID, "unknown flags 0x%x", p->flags);
  const uint32_t variant = p->flags & (BDRS_F_OLD_KERNEL | BDRS_F_NO_MOMENTUM | BDRS_F_DEBIASED);
  if (variant && p->lambda != 1.0) return fail(BDRS_E_INVALID, "the ablation variant flags need lambda = 1");
  if ((variant & BDRS_F_DEBIASED) && (variant & (BDRS_F_OLD_KERNEL | BDRS_F_NO_MOMENTUM)) !=
                                         (BDRS_F_OLD_KERNEL | BDRS_F_NO_MOMENTUM))
    return fail(BDRS_E_INVALID, "flags: BDRS_F_DEBIASED needs BDRS_F_OLD_KERNEL and BDRS_F_NO_MOMENTUM");
  if (!p->workspace) return fail(BDRS_E_INVALID, "workspace is NULL");
  if (((uintptr_t)p->workspace) % kAlign) return fail(BDRS_E_INVALID, "workspace must be 256-byte aligned");
  if (need == 0) need = make_layout(p->m, p->n, p->dim, 0, 0, (p->flags & BDRS_F_KEEP_BEST_STATE) != 0).total;
  if (p->workspace_bytes < need)
    return fail(BDRS_E_NOMEM, "workspace too small: %zu bytes given, %zu needed", p->workspace_bytes, need);
  return BDRS_OK;
}

bdrs_status check_device() {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count < 1) return fail(BDRS_E_DEVICE, "no HIP device available");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(BDRS_E_DEVICE, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
  return BDRS_OK;
}

// 21-bit-per-axis Morton code of a point quantised over the side's bounding box.
uint64_t spread3(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffull;
  v = (v | v << 16) & 0x1f0000ff0000ffull;
  v = (v | v << 8) & 0x100f00f00f00f00full;
  v = (v | v << 4) & 0x10c30c30c30c30c3ull;
  v = (v | v << 2) & 0x1249249249249249ull;
  return v;
}
uint64_t spread2(uint64_t v) {
  v &= 0xffffffffull;
  v = (v | v << 16) & 0x0000ffff0000ffffull;
  v = (v | v << 8) & 0x00ff00ff00ff00ffull;
  v = (v | v << 4) & 0x0f0f0f0f0f0f0f0full;
  v = (v | v << 2) & 0x3333333333333333ull;
  v = (v | v << 1) & 0x5555555555555555ull;
  return v;
}

void build_side(const float* pts, const double* w, int count, int dim, const double origin[3], const SideShape& sh,
                HostSide& hs) {
  // tile order: Morton order of the quantised coordinates
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < dim; ++d) {
    lo[d] = hi[d] = pts[d];
    for (int i = 0; i < count; ++i) {
      lo[d] = std::min(lo[d], (double)pts[(size_t)i * dim + d]);
      hi[d] = std::max(hi[d], (double)pts[(size_t)i * dim + d]);
    }
  }
  const int bits = dim == 1 ? 31 : (dim == 2 ? 31 : 21);
  const double qmax = (double)((1u << bits) - 1);
  std::vector<uint64_t> code(count);
  for (int i = 0; i < count; ++i) {
    uint64_t q[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
      const double span = hi[d] - lo[d];
      q[d] = span > 0 ? (uint64_t)std::llround((pts[(size_t)i * dim + d] - lo[d]) / span * qmax) : 0;
    }
    code[i] = dim == 1 ? q[0] : (dim == 2 ? (spread2(q[0]) | spread2(q[1]) << 1)
                                          : (spread3(q[0]) | spread3(q[1]) << 1 | spread3(q[2]) << 2));
  }
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return code[a] < code[b]; });

  hs.perm.assign(sh.np, order[count - 1]);
  hs.iperm.assign(count, 0);
  for (int s = 0; s < count; ++s) {
    hs.perm[s] = order[s];
    hs.iperm[order[s]] = s;
  }
  hs.abs.assign((size_t)dim * sh.np, 0.f);
  for (int s = 0; s < sh.np; ++s) {
    const int i = hs.perm[s];
    for (int d = 0; d < dim; ++d) hs.abs[(size_t)d * sh.np + s] = (float)((double)pts[(size_t)i * dim + d] - origin[d]);
  }
  hs.marg.assign(sh.np, 0.0);
  hs.logm.assign(sh.np, -INFINITY);
  for (int s = 0; s < count; ++s) {
    hs.marg[s] = w[hs.perm[s]];
    hs.logm[s] = std::log(w[hs.perm[s]]);
  }
  hs.off.assign((size_t)sh.ntiles * dim * kTile, 0.f);
  TileRec blank{};
  blank.amax = -INFINITY;
  blank.alpha = -INFINITY;
  hs.tile.assign((size_t)sh.ntiles, blank);
  for (int t = 0; t < sh.ntiles; ++t) {
    const int s0 = t * kTile, s1 = std::min(count, s0 + kTile);
    for (int d = 0; d < dim; ++d) {
      float mn = hs.abs[(size_t)d * sh.np + s0], mx = mn;
      for (int s = s0; s < s1; ++s) {
        mn = std::min(mn, hs.abs[(size_t)d * sh.np + s]);
        mx = std::max(mx, hs.abs[(size_t)d * sh.np + s]);
      }
      const float ctr = 0.5f * (mn + mx);
      float rad = 0.f;
      for (int s = s0; s < s0 + kTile; ++s) {
        const float b = hs.abs[(size_t)d * sh.np + s] - ctr;
        hs.off[((size_t)t * dim + d) * kTile + (s - s0)] = b;
        if (s < s1) rad = std::max(rad, std::fabs(b));
      }
      hs.tile[t].ctr[d] = ctr;
      hs.tile[t].rad[d] = rad;
    }
  }
  // geometry of each tile's real points for the epilogues' plane fits, from
  // the float32 offsets the device holds
  hs.geom.assign((size_t)sh.ntiles, TileGeom{});
  for (int t = 0; t < sh.ntiles; ++t) {
    TileGeom& g = hs.geom[t];
    const int s0 = t * kTile, n = std::min(count, s0 + kTile) - s0;
    auto b = [&](int q, int d) { return (double)hs.off[((size_t)t * dim + d) * kTile + q]; };
    g.cnt = (double)n;
    for (int d = 0; d < dim; ++d) {
      double s = 0.0;
      for (int q = 0; q < n; ++q) s += b(q, d);
      g.mb[d] = s / n;
    }
    double c[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int q = 0; q < n; ++q)
      for (int d = 0; d < dim; ++d)
        for (int e = 0; e < dim; ++e) c[d][e] += (b(q, d) - g.mb[d]) * (b(q, e) - g.mb[e]);
    // inverse by cofactors; a (near-)singular matrix keeps the plane flat
    double inv[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if (dim == 1) {
      if (c[0][0] > 1e-12) inv[0][0] = 1.0 / c[0][0];
    } else if (dim == 2) {
      const double det = c[0][0] * c[1][1] - c[0][1] * c[1][0];
      if (std::fabs(det) > 1e-12 * (c[0][0] * c[1][1] + 1e-300)) {
        inv[0][0] = c[1][1] / det;
        inv[1][1] = c[0][0] / det;
        inv[0][1] = inv[1][0] = -c[0][1] / det;
      }
    } else {
      const double a00 = c[1][1] * c[2][2] - c[1][2] * c[2][1];
      const double a01 = c[0][2] * c[2][1] - c[0][1] * c[2][2];
      const double a02 = c[0][1] * c[1][2] - c[0][2] * c[1][1];
      const double det = c[0][0] * a00 + c[1][0] * a01 + c[2][0] * a02;
      if (std::fabs(det) > 1e-12 * (c[0][0] * c[1][1] * c[2][2] + 1e-300)) {
        inv[0][0] = a00 / det;
        inv[0][1] = inv[1][0] = a01 / det;
        inv[0][2] = inv[2][0] = a02 / det;
        inv[1][1] = (c[0][0] * c[2][2] - c[0][2] * c[2][0]) / det;
        inv[1][2] = inv[2][1] = (c[0][2] * c[1][0] - c[0][0] * c[1][2]) / det;
        inv[2][2] = (c[0][0] * c[1][1] - c[0][1] * c[1][0]) / det;
      }
    }
    g.cinv[0] = inv[0][0];
    g.cinv[1] = inv[0][1];
    g.cinv[2] = inv[0][2];
    g.cinv[3] = inv[1][1];
    g.cinv[4] = inv[1][2];
    g.cinv[5] = inv[2][2];
  }
}



void fill_ctx(bdrs_solver s) {
  const Layout& L = s->L;
  char* base = (char*)s->prm.workspace;
  LaunchCtx& c = s->ctx;
  c.stream = (hipStream_t)s->prm.stream;
  c.dim = s->prm.dim;
  c.splits_row = L.splits_row;
  c.splits_col = L.splits_col;
  c.ctrl = (Ctrl*)(base + L.ctrl);
  auto side = [&](SideDev& sd, const SideShape& sh, size_t abs, size_t off, size_t tile, size_t geom, size_t A,
                  size_t perm, size_t marg, size_t logm, size_t iperm, size_t hint) {
    sd.count = sh.count;
    sd.ntiles = sh.ntiles;
    sd.np = sh.np;
    sd.pad = 0;
    sd.abs = (float*)(base + abs);
    sd.off = (float*)(base + off);
    sd.tile = (TileRec*)(base + tile);
    sd.geom = (const TileGeom*)(base + geom);
    sd.A = (float*)(base + A);
    sd.perm = (int*)(base + perm);
    sd.marg = (double*)(base + marg);
    sd.logmarg = (double*)(base + logm);
    sd.iperm = (int*)(base + iperm);
    sd.hint = (int*)(base + hint);
  };
  side(c.rows, L.R, L.r_abs, L.r_off, L.r_tile, L.r_geom, L.r_A, L.r_perm, L.r_marg, L.r_logm, L.r_iperm,
       L.r_hint);
  side(c.cols, L.C, L.c_abs, L.c_off, L.c_tile, L.c_geom, L.c_A, L.c_perm, L.c_marg, L.c_logm, L.c_iperm,
       L.c_hint);
  c.st.la = (double*)(base + L.la);
  c.st.lah = (double*)(base + L.lah);
  c.st.lb1 = (double*)(base + L.lb1);
  c.st.lb2 = (double*)(base + L.lb2);
  c.st.lbh = (double*)(base + L.lbh);
  c.st.lt[0] = (double*)(base + L.lt0);
  c.st.lt[1] = (double*)(base + L.lt1);
  c.st.mu = (double*)(base + L.mu);
  c.st.logs = (double*)(base + L.logs);
  c.st.pvec = (double*)(base + L.pvec);
  c.part.rec = (void*)(base + L.part);
  c.part.ref = (double*)(base + L.part_ref);
  c.part.splits = L.splits_max;
  c.cert_part = (double*)(base + L.cert_part);
  c.cert_out = (double*)(base + L.cert_out);
  c.cert_blocks = L.cert_blocks;
  c.plan_row = (double*)(base + L.plan_row);
  c.plan_col = (double*)(base + L.plan_col);
  c.plan_aux = (double*)(base + L.plan_aux);
  c.plan_stats = (double*)(base + L.plan_stats);
  c.tile_count = nullptr;  // set for profiled sweeps only
  c.tile_total = nullptr;
  c.ev_start = nullptr;
  c.ev_stop = nullptr;
}

// reads the device iteration counter (synchronises the stream)
bdrs_status sync_k(bdrs_solver s) {
  long long k = 0;
  HIPCHK(hipMemcpyAsync(&k, &s->ctx.ctrl->k, sizeof k, hipMemcpyDeviceToHost, s->ctx.stream));
  HIPCHK(hipStreamSynchronize(s->ctx.stream));
  s->k = k;
  return BDRS_OK;
}

double eps_at(const bdrs_solver s, long long k) { return s->prm.eta / (s->prm.lambda * (double)k + 1.0); }

// temperature of the row update of iteration k (the certificate's plan uses it)
double eps_row_at(const bdrs_solver s, long long k) {
  if (s->prm.flags & BDRS_F_OLD_KERNEL) return k >= 1 ? s->prm.eta / (double)k : s->prm.eta * kFarTemperature;
  return eps_at(s, k);
}

// variants whose certificate plan differs from the fused column statistics
bool separate_cert(const bdrs_solver s) { return (s->prm.flags & (BDRS_F_OLD_KERNEL | BDRS_F_DEBIASED)) != 0; }

bdrs_status hip_status(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(BDRS_E_DEVICE, "HIP error %s in %s", hipGetErrorString(e), what);
  return BDRS_OK;
}

// one LSE sweep launch, bracketed by HIP events when profiling is on; a
// profiled sweep also counts the input tiles its wavefronts evaluated
hipError_t sweep(bdrs_solver s, bool transpose, bool cert, int splits, double eps_arg, int kofs = 0) {
  if (!s->prof) return launch_sweep(s->ctx, transpose, cert, splits, eps_arg, kofs);
  while (s->ev_pool.size() < s->ev_used + 2) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    s->ev_pool.push_back(ev);
  }
  char* base = (char*)s->prm.workspace;
  LaunchCtx c = s->ctx;
  c.tile_count = (unsigned*)(base + s->L.tile_count);
  c.tile_total = (unsigned long long*)(base + s->L.tile_total);
  // the launch records the events at the kernel's own start and end
  c.ev_start = s->ev_pool[s->ev_used];
  c.ev_stop = s->ev_pool[s->ev_used + 1];
  hipError_t e = launch_sweep(c, transpose, cert, splits, eps_arg, kofs);
  const int np_out = transpose ? c.cols.np : c.rows.np;
  if (e == hipSuccess) e = launch_count_tiles(c, splits * (np_out / kTile));
  if (e == hipSuccess) {
    s->ev_used += 2;
    s->prof_sweeps += 1;
    s->prof_entries += (double)s->prm.m * (double)s->prm.n;
  }
  return e;
}

// one iteration of Algorithm 1; with cert the column sweep also gathers Algorithm 2's statistics
bdrs_status enqueue_iteration(bdrs_solver s, bool cert, int kofs) {
  const LaunchCtx& c = s->ctx;
  hipError_t e;
  if ((e = sweep(s, false, false, s->L.splits_row, -1.0, kofs)) != hipSuccess) return hip_status(e, "row sweep");
  if ((e = launch_finish(c, false, kFinishRow, s->L.splits_row, -1.0, nullptr, kofs)) != hipSuccess)
    return hip_status(e, "row finish");
  if ((e = sweep(s, true, cert, s->L.splits_col, -1.0, kofs)) != hipSuccess) return hip_status(e, "col sweep");
  if ((e = launch_finish(c, true, cert ? kFinishColCert : kFinishCol, s->L.splits_col, -1.0, nullptr, kofs)) !=
      hipSuccess)
    return hip_status(e, "col finish");
  s->packed_rows = true;
  return BDRS_OK;
}

// re-derives the packed sweep weights from the dual state (after bdrs_lse or a repair pass)
bdrs_status repack(bdrs_solver s) {
  const LaunchCtx& c = s->ctx;
  hipError_t e;
  if ((e = launch_prologue(c)) != hipSuccess) return hip_status(e, "prologue");
  if (s->k > 0) {
    // rows.A <- log alpha-hat of iteration k-1 with that iteration's temperature
    if ((e = launch_pack_rows_from_lah(c, eps_row_at(s, s->k - 1))) != hipSuccess) return hip_status(e, "repack");
    s->packed_rows = true;
  }
  return BDRS_OK;
}

// certificate record (kCertSlots doubles, host) -> bdrs_cert, updating the best bounds
// Copies the dual state and the hints into the retained-state region
// (to_best) or back, on the solver's stream (device to device, tile order).
hipError_t copy_best(bdrs_solver s, bool to_best) {
  const LaunchCtx& c = s->ctx;
  char* base = (char*)s->prm.workspace;
  const size_t nr = sizeof(double) * c.rows.np, nc = sizeof(double) * c.cols.np;
  struct Pair {
    void* live;
    size_t best, bytes;
  } pairs[] = {
      {c.st.la, s->L.best_la, nr},   {c.st.lah, s->L.best_lah, nr}, {c.st.lb1, s->L.best_lb1, nc},
      {c.st.lb2, s->L.best_lb2, nc}, {c.st.lbh, s->L.best_lbh, nc}, {c.st.lt[0], s->L.best_lt0, nc},
      {c.st.lt[1], s->L.best_lt1, nc}, {c.rows.hint, s->L.best_hr, sizeof(int) * c.rows.np},
      {c.cols.hint, s->L.best_hc, sizeof(int) * c.cols.np},
  };
  hipError_t e = hipSuccess;
  for (const Pair& q : pairs) {
    void* b = base + q.best;
    if (e == hipSuccess)
      e = hipMemcpyAsync(to_best ? b : q.live, to_best ? q.live : b, q.bytes, hipMemcpyDeviceToDevice, c.stream);
  }
  return e;
}

bdrs_status cert_from_record(bdrs_solver s, const double* h, bool repair, bdrs_cert* out) {
  // Prop. 3 gives L <= p* <= U for every certificate, hence also
  // U_best = min U >= p* >= max L = L_best; a computed gap below this
  // tolerance (relative to U) contradicts it and invalidates the bounds.
  constexpr double kNegGapTol = 1e-9;
  bdrs_cert ce;
  ce.k = (int64_t)h[0];
  ce.eps = h[1];
  ce.L = h[2];
  ce.U = h[3];
  ce.delta = h[4];
  ce.cost_Z = h[5];
  ce.n_nonfinite = (int64_t)h[7];
  ce.gap = ce.U - ce.L;
  ce.rel_gap = ce.U > 1e-300 ? ce.gap / ce.U : ce.gap;
  ce.repaired_cost = repair ? h[8] : NAN;
  const bool finite = ce.n_nonfinite == 0 && std::isfinite(ce.L) && std::isfinite(ce.U);
  const bool neg_own = ce.gap < -kNegGapTol * std::fabs(ce.U);
  if (finite && !neg_own) {  // an invalid certificate is not folded into the best bounds
    if (ce.U < s->U_best) {
      s->U_best = ce.U;
      s->kU = ce.k;
    }
    if (ce.L > s->L_best) {
      s->L_best = ce.L;
      s->kL = ce.k;
    }
  }
  ce.U_best = s->U_best;
  ce.L_best = s->L_best;
  ce.k_U_best = s->kU;
  ce.k_L_best = s->kL;
  const double g = s->U_best - s->L_best;
  ce.rel_gap_best = s->U_best > 1e-300 ? g / s->U_best : g;
  const bool neg_best = std::isfinite(g) && g < -kNegGapTol * std::fabs(s->U_best);
  ce.negative_gap = (neg_own || neg_best) ? 1 : 0;
  if (out) *out = ce;
  if (!finite)
    return fail(BDRS_E_NUMERIC, "non-finite values in the certificate at iteration %lld", (long long)ce.k);
  if (ce.negative_gap)
    return fail(BDRS_E_NUMERIC,
                "negative duality gap at iteration %lld: U - L = %.6e, U_best - L_best = %.6e "
                "(Prop. 3 gives L <= p* <= U: float32 error in the sweeps or omega below osc(C))",
                (long long)ce.k, ce.gap, g);
  if (s->L.keep_best && ce.rel_gap < s->best_rel) {
    // the state after iteration k (the certified one) becomes the retained state
    const hipError_t e = copy_best(s, true);
    if (e != hipSuccess) return hip_status(e, "keep best state");
    s->best_rel = ce.rel_gap;
    s->best_k = ce.k + 1;
  }
  return BDRS_OK;
}

bdrs_status read_cert(bdrs_solver s, bool repair, bdrs_cert* out) {
  double h[kCertSlots];
  HIPCHK(hipMemcpyAsync(h, s->ctx.cert_out, sizeof h, hipMemcpyDeviceToHost, s->ctx.stream));
  HIPCHK(hipStreamSynchronize(s->ctx.stream));
  return cert_from_record(s, h, repair, out);
}

// Algorithm 2's column statistics of the last finished iteration by a separate
// column sweep: the plan Z = diag(alpha-hat) K diag(t) at the row update's
// temperature (rows re-packed from log alpha-hat when the last row epilogue
// packed other weights or another temperature).
bdrs_status enqueue_cert_only(bdrs_solver s) {
  bdrs_status st;
  if ((!s->packed_rows || separate_cert(s)) && (st = repack(s)) != BDRS_OK) return st;
  const LaunchCtx& c = s->ctx;
  const double eps = eps_row_at(s, s->k - 1);
  hipError_t e;
  if ((e = sweep(s, true, true, s->L.splits_col, eps)) != hipSuccess) return hip_status(e, "cert sweep");
  if ((e = launch_finish(c, true, kFinishCertOnly, s->L.splits_col, eps, nullptr, 0)) != hipSuccess)
    return hip_status(e, "cert finish");
  return BDRS_OK;
}

bdrs_status enqueue_repair(bdrs_solver s) {
  const LaunchCtx& c = s->ctx;
  hipError_t e;
  const double eps = eps_row_at(s, s->k - 1);
  if ((e = launch_repair_pack(c)) != hipSuccess) return hip_status(e, "repair pack");
  if ((e = sweep(s, false, false, s->L.splits_row, eps)) != hipSuccess) return hip_status(e, "repair sweep");
  if ((e = launch_finish(c, false, kFinishRepair, s->L.splits_row, eps, nullptr, 0)) != hipSuccess)
    return hip_status(e, "repair finish");
  if ((e = launch_repair_reduce(c)) != hipSuccess) return hip_status(e, "repair reduce");
  if ((e = launch_prologue(c)) != hipSuccess) return hip_status(e, "prologue");  // restore cols.A
  return BDRS_OK;
}

size_t row_sweep_items(const Layout& L) { return (size_t)(L.R.np / kSweepBlock) * L.splits_row; }
size_t col_sweep_items(const Layout& L) { return (size_t)(L.C.np / kSweepBlock) * L.splits_col; }

BatchLayout batch_layout(const std::vector<const Layout*>& ls) {
  BatchLayout B{};
  for (const Layout* L : ls) {
    B.n_rs += row_sweep_items(*L);
    B.n_cs += col_sweep_items(*L);
    B.n_rf += L->R.ntiles;
    B.n_cf += L->C.ntiles;
    B.n_ce += L->cert_blocks;
  }
  const size_t count = ls.size();
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  B.descs = take(sizeof(LaunchCtx) * count);
  B.items_rs = take(sizeof(BatchItem) * B.n_rs);
  B.items_cs = take(sizeof(BatchItem) * B.n_cs);
  B.items_rf = take(sizeof(BatchItem) * B.n_rf);
  B.items_cf = take(sizeof(BatchItem) * B.n_cf);
  B.items_ce = take(sizeof(BatchItem) * B.n_ce);
  B.probs = take(sizeof(int) * count);
  B.records = take(sizeof(double) * kCertSlots * count);
  B.total = o;
  return B;
}

std::vector<const Layout*> layouts_of(const std::vector<bdrs_solver>& members) {
  std::vector<const Layout*> ls;
  for (bdrs_solver s : members) ls.push_back(&s->L);
  return ls;
}

size_t BatchEngine::bytes_for(const std::vector<bdrs_solver>& members) { return batch_layout(layouts_of(members)).total; }
size_t BatchEngine::bytes_for_layouts(const std::vector<const Layout*>& layouts) {
  return batch_layout(layouts).total;
}

BatchEngine::~BatchEngine() {
  if (exec_) (void)hipGraphExecDestroy(exec_);  // teardown: nothing to report
}

hipError_t BatchEngine::bind(const std::vector<bdrs_solver>& members, char* ws, int block_iters, bool use_graph,
                             hipStream_t st) {
  if (exec_) {
    (void)hipGraphExecDestroy(exec_);
    exec_ = nullptr;
  }
  members_ = members;
  ws_ = ws;
  st_ = st;
  iters_ = block_iters;
  B_ = batch_layout(layouts_of(members_));
  dim_ = members_.empty() ? 0 : members_[0]->prm.dim;
  std::vector<LaunchCtx> descs;
  std::vector<BatchItem> rs, cs, rf, cf, ce;
  std::vector<int> probs;
  for (int p = 0; p < (int)members_.size(); ++p) {
    const bdrs_solver s = members_[p];
    descs.push_back(s->ctx);
    // split fastest: consecutive items go to consecutive XCDs, so an output
    // block's splits spread over the XCDs (as in the single-problem launch)
    for (int b = 0; b < s->L.R.np / kSweepBlock; ++b)
      for (int sp = 0; sp < s->L.splits_row; ++sp) rs.push_back({p, b, sp, 0});
    for (int b = 0; b < s->L.C.np / kSweepBlock; ++b)
      for (int sp = 0; sp < s->L.splits_col; ++sp) cs.push_back({p, b, sp, 0});
    for (int t = 0; t < s->L.R.ntiles; ++t) rf.push_back({p, t, 0, 0});
    for (int t = 0; t < s->L.C.ntiles; ++t) cf.push_back({p, t, 0, 0});
    for (int b = 0; b < s->L.cert_blocks; ++b) ce.push_back({p, b, 0, 0});
    probs.push_back(p);
  }
  nrs_ = (int)rs.size();
  ncs_ = (int)cs.size();
  nrf_ = (int)rf.size();
  ncf_ = (int)cf.size();
  nce_ = (int)ce.size();
  hipError_t r = hipSuccess;
  auto up = [&](size_t off, const void* src, size_t bytes) {
    if (r == hipSuccess && bytes) r = hipMemcpyAsync(ws_ + off, src, bytes, hipMemcpyHostToDevice, st_);
  };
  up(B_.descs, descs.data(), descs.size() * sizeof(LaunchCtx));
  up(B_.items_rs, rs.data(), rs.size() * sizeof(BatchItem));
  up(B_.items_cs, cs.data(), cs.size() * sizeof(BatchItem));
  up(B_.items_rf, rf.data(), rf.size() * sizeof(BatchItem));
  up(B_.items_cf, cf.data(), cf.size() * sizeof(BatchItem));
  up(B_.items_ce, ce.data(), ce.size() * sizeof(BatchItem));
  up(B_.probs, probs.data(), probs.size() * sizeof(int));
  if (r == hipSuccess) r = hipStreamSynchronize(st_);  // host vectors go out of scope
  if (r == hipSuccess && use_graph) r = capture();
  return r;
}

hipError_t BatchEngine::capture() {
  if (exec_ || members_.empty()) return hipSuccess;
  hipGraph_t g = nullptr;
  hipError_t r = hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal);
  if (r == hipSuccess) {
    const hipError_t r2 = enqueue(st_);
    r = hipStreamEndCapture(st_, &g);
    if (r == hipSuccess) r = r2;
  }
  if (r == hipSuccess) r = hipGraphInstantiate(&exec_, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (r != hipSuccess) exec_ = nullptr;
  return r;
}

// one block of iters_ iterations (the last with the fused certificate) plus
// the certificate reductions of every member
hipError_t BatchEngine::enqueue(hipStream_t st) {
  const LaunchCtx* descs = (const LaunchCtx*)(ws_ + B_.descs);
  const BatchItem* rs = (const BatchItem*)(ws_ + B_.items_rs);
  const BatchItem* cs = (const BatchItem*)(ws_ + B_.items_cs);
  const BatchItem* rf = (const BatchItem*)(ws_ + B_.items_rf);
  const BatchItem* cf = (const BatchItem*)(ws_ + B_.items_cf);
  const BatchItem* ce = (const BatchItem*)(ws_ + B_.items_ce);
  hipError_t e = hipSuccess;
  for (int i = 0; i < iters_ && e == hipSuccess; ++i) {
    const bool cert = (i == iters_ - 1);
    e = launch_sweep_batch(rs, nrs_, descs, dim_, false, false, i, st);
    if (e == hipSuccess) e = launch_finish_batch(rf, nrf_, descs, false, kFinishRow, i, st);
    if (e == hipSuccess) e = launch_sweep_batch(cs, ncs_, descs, dim_, true, cert, i, st);
    if (e == hipSuccess) e = launch_finish_batch(cf, ncf_, descs, true, cert ? kFinishColCert : kFinishCol, i, st);
  }
  if (e == hipSuccess) e = launch_advance_batch(descs, (int)members_.size(), iters_, st);
  if (e == hipSuccess)
    e = launch_cert_batch(ce, nce_, (const int*)(ws_ + B_.probs), (int)members_.size(), descs,
                          (double*)(ws_ + B_.records), st);
  return e;
}

hipError_t BatchEngine::run_block() {
  if (members_.empty()) return hipSuccess;
  return exec_ ? hipGraphLaunch(exec_, st_) : enqueue(st_);
}

hipError_t BatchEngine::read_records(std::vector<double>& rec) {
  rec.resize(members_.size() * kCertSlots);
  if (rec.empty()) return hipSuccess;
  hipError_t e = hipMemcpyAsync(rec.data(), ws_ + B_.records, rec.size() * sizeof(double), hipMemcpyDeviceToHost, st_);
  if (e == hipSuccess) e = hipStreamSynchronize(st_);
  return e;
}

bdrs_status check_batch(const bdrs_solver* sv, int count) {
  if (!sv) return fail(BDRS_E_INVALID, "solvers is NULL");
  if (count < 1) return fail(BDRS_E_INVALID, "count must be >= 1");
  for (int i = 0; i < count; ++i) {
    if (!sv[i]) return fail(BDRS_E_INVALID, "solvers[%d] is NULL", i);
    if (sv[i]->prm.dim != sv[0]->prm.dim) return fail(BDRS_E_INVALID, "solvers[%d] has another dim", i);
    for (int j = 0; j < i; ++j)
      if (sv[j] == sv[i]) return fail(BDRS_E_INVALID, "solvers[%d] is listed twice", i);
  }
  return BDRS_OK;
}

}  // namespace bdrs_host

using namespace bdrs_host;

extern "C" {

bdrs_status bdrs_batch_workspace_size(const bdrs_solver* solvers, int32_t count, size_t* bytes) {
  bdrs_status st = check_batch(solvers, count);
  if (st != BDRS_OK) return st;
  if (!bytes) return fail(BDRS_E_INVALID, "bytes is NULL");
  *bytes = BatchEngine::bytes_for(std::vector<bdrs_solver>(solvers, solvers + count));
  return BDRS_OK;
}

}  // extern "C"

namespace bdrs_host {

// Host checks shared by the batched entry points (no device work except
// reading each solver's iteration counter); need: the work-list bytes.
bdrs_status check_batch_call(const bdrs_solver* solvers, int32_t count, double tau, int32_t max_iters,
                             int32_t cert_every, const bdrs_cert* outs, const int32_t* statuses, size_t* need) {
  bdrs_status st = check_batch(solvers, count);
  if (st != BDRS_OK) return st;
  if (!outs || !statuses) return fail(BDRS_E_INVALID, "outs and statuses are required");
  if (!(tau >= 0 && std::isfinite(tau))) return fail(BDRS_E_INVALID, "tau must be finite and >= 0");
  if (cert_every < 1) return fail(BDRS_E_INVALID, "cert_every must be >= 1");
  if (max_iters < 1 || max_iters % cert_every)
    return fail(BDRS_E_INVALID, "max_iters must be a positive multiple of cert_every");
  *need = BatchEngine::bytes_for(std::vector<bdrs_solver>(solvers, solvers + count));
  return BDRS_OK;
}

bdrs_status check_batch_members(const bdrs_solver* solvers, int32_t count, int32_t cert_every) {
  bdrs_status st;
  for (int i = 0; i < count; ++i) {
    if ((st = sync_k(solvers[i])) != BDRS_OK) return st;
    if (solvers[i]->k % cert_every)
      return fail(BDRS_E_STATE, "solvers[%d] is at iteration %lld, not a multiple of cert_every", i, solvers[i]->k);
    if (solvers[i]->prm.flags & BDRS_F_REPAIR)
      return fail(BDRS_E_INVALID, "solvers[%d]: BDRS_F_REPAIR is not supported in batches", i);
    if (separate_cert(solvers[i]))
      return fail(BDRS_E_INVALID, "solvers[%d]: old-kernel and debiased variants are not batched", i);
    if (solvers[i]->L.keep_best)
      return fail(BDRS_E_INVALID, "solvers[%d]: BDRS_F_KEEP_BEST_STATE is not supported in batches", i);
  }
  return BDRS_OK;
}

// The block loop of a batched solve on stream st_b with the work lists in ws;
// synchronises st_b before it returns.
bdrs_status run_batch(const bdrs_solver* solvers, int32_t count, char* ws, double tau, int32_t tau_relative,
                      int32_t max_iters, int32_t cert_every, bool use_graph, hipStream_t st_b, bdrs_cert* outs,
                      int32_t* statuses) {
  std::vector<bdrs_solver> all(solvers, solvers + count);
  std::vector<int> index(count), done_iters(count, 0);
  for (int i = 0; i < count; ++i) {
    index[i] = i;
    statuses[i] = BDRS_NOT_CONVERGED;
  }
  std::vector<int> active = index;
  bdrs_status result = BDRS_OK;
  hipError_t e;
  {
    BatchEngine eng;
    e = eng.bind(all, ws, cert_every, use_graph, st_b);
    std::vector<double> rec;
    while (e == hipSuccess && !active.empty()) {
      e = eng.run_block();
      if (e == hipSuccess) e = eng.read_records(rec);
      if (e != hipSuccess) break;
      std::vector<int> still;
      for (size_t q = 0; q < active.size(); ++q) {
        const int p = active[q];
        bdrs_solver s = solvers[p];
        s->k += cert_every;
        done_iters[p] += cert_every;
        const bdrs_status cs_st = cert_from_record(s, rec.data() + q * kCertSlots, false, &outs[p]);
        const double target = tau_relative ? outs[p].rel_gap_best : (outs[p].U_best - outs[p].L_best);
        if (cs_st != BDRS_OK) {
          statuses[p] = cs_st;
          result = cs_st;
        } else if (target <= tau) {
          statuses[p] = BDRS_OK;
        } else if (done_iters[p] >= max_iters) {
          statuses[p] = BDRS_NOT_CONVERGED;
          if (result == BDRS_OK) result = BDRS_NOT_CONVERGED;
        } else {
          still.push_back(p);
        }
      }
      if (still.size() != active.size()) {
        active.swap(still);
        std::vector<bdrs_solver> mem;
        for (int p : active) mem.push_back(solvers[p]);
        e = eng.bind(mem, ws, cert_every, use_graph, st_b);
      }
    }
  }
  const hipError_t es = hipStreamSynchronize(st_b);  // also reports a fault of the last block
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return fail(BDRS_E_DEVICE, "HIP error %s in batch solve", hipGetErrorString(e));
  for (int i = 0; i < count; ++i) solvers[i]->packed_rows = true;
  return result;
}

// Device storage of bdrs_batch_solve_static: one array on every GPU the
// library runs on, held until the process ends.  In host code `scratch` only
// stands in for the symbol; its address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is handed to copies and kernels.
static __device__ __align__(256) char scratch[BDRS_BATCH_STATIC_BYTES];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_addr;  // device -> address of its `scratch`

// Address of the current device's array (looked up on the first call there).
bdrs_status static_scratch(char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(BDRS_E_DEVICE, "HIP error %s taking the address of the static batch array on device %d",
                  hipGetErrorString(e), dev);
    it = g_scratch_addr.emplace(dev, (char*)ptr).first;
  }
  *out = it->second;
  return BDRS_OK;
}

}  // namespace bdrs_host

extern "C" {

bdrs_status bdrs_batch_solve_static(const bdrs_solver* solvers, int32_t count, double tau, int32_t tau_relative,
                                    int32_t max_iters, int32_t cert_every, bdrs_cert* outs, int32_t* statuses) {
  size_t need = 0;
  bdrs_status st = check_batch_call(solvers, count, tau, max_iters, cert_every, outs, statuses, &need);
  if (st != BDRS_OK) return st;
  if (need > (size_t)BDRS_BATCH_STATIC_BYTES)
    return fail(BDRS_E_NOMEM, "the batch needs %zu bytes of work lists, the static array holds %zu", need,
                (size_t)BDRS_BATCH_STATIC_BYTES);
  if ((st = check_batch_members(solvers, count, cert_every)) != BDRS_OK) return st;
  char* ws = nullptr;
  if ((st = static_scratch(&ws)) != BDRS_OK) return st;
  // the first solver's stream; no graph (instantiating one allocates)
  return run_batch(solvers, count, ws, tau, tau_relative, max_iters, cert_every, false, solvers[0]->ctx.stream, outs,
                   statuses);
}

bdrs_status bdrs_batch_solve(const bdrs_solver* solvers, int32_t count, void* workspace, size_t workspace_bytes,
                             double tau, int32_t tau_relative, int32_t max_iters, int32_t cert_every,
                             int32_t use_graph, bdrs_cert* outs, int32_t* statuses) {
  size_t need = 0;
  bdrs_status st = check_batch_call(solvers, count, tau, max_iters, cert_every, outs, statuses, &need);
  if (st != BDRS_OK) return st;
  if (!workspace || ((uintptr_t)workspace) % kAlign)
    return fail(BDRS_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
  if (workspace_bytes < need)
    return fail(BDRS_E_NOMEM, "batch workspace too small: %zu bytes given, %zu needed", workspace_bytes, need);
  if ((st = check_batch_members(solvers, count, cert_every)) != BDRS_OK) return st;
  hipStream_t st_b = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&st_b, hipStreamNonBlocking));
  st = run_batch(solvers, count, (char*)workspace, tau, tau_relative, max_iters, cert_every, use_graph != 0, st_b,
                 outs, statuses);
  (void)hipStreamDestroy(st_b);
  return st;
}

const char* bdrs_last_error(void) { return g_err.c_str(); }

const char* bdrs_version(void) { return "bdrs-gfx950 0.1"; }

bdrs_status bdrs_workspace_size(const bdrs_params* p, size_t* bytes) {
  bdrs_status st = check_sizes(p);
  if (st != BDRS_OK) return st;
  if (!bytes) return fail(BDRS_E_INVALID, "bytes is NULL");
  *bytes = make_layout(p->m, p->n, p->dim, 0, 0, (p->flags & BDRS_F_KEEP_BEST_STATE) != 0).total;
  return BDRS_OK;
}

bdrs_status bdrs_create(const bdrs_params* p, bdrs_solver* out) {
  if (!out) return fail(BDRS_E_INVALID, "out is NULL");
  *out = nullptr;
  bdrs_status st = check_params(p);
  if (st != BDRS_OK) return st;
  if ((st = check_device()) != BDRS_OK) return st;

  std::vector<float> hx, hy;
  std::vector<double> hr, hc;
  if ((st = download_inputs(p, hx, hy, hr, hc)) != BDRS_OK) return st;
  return create_from_host(p, hx.data(), hy.data(), hr.data(), hc.data(), out);
}

}  // extern "C"

namespace bdrs_host {

bdrs_status download_inputs(const bdrs_params* p, std::vector<float>& hx, std::vector<float>& hy,
                            std::vector<double>& hr, std::vector<double>& hc) {
  const int m = p->m, n = p->n, dim = p->dim;
  hipStream_t stream = (hipStream_t)p->stream;
  hx.resize((size_t)m * dim);
  hy.resize((size_t)n * dim);
  hr.resize(m);
  hc.resize(n);
  HIPCHK(hipMemcpyAsync(hx.data(), p->x, hx.size() * sizeof(float), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(hy.data(), p->y, hy.size() * sizeof(float), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(hr.data(), p->r, m * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(hc.data(), p->c, n * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return BDRS_OK;
}

bdrs_status prepare_image(const bdrs_params* p, const float* px, const float* py, const double* pr, const double* pc,
                          HostImage& img) {
  const int m = p->m, n = p->n, dim = p->dim;
  // contents: finite coordinates, strictly positive marginals of unit mass (Eq. 1)
  for (size_t i = 0; i < (size_t)m * dim; ++i)
    if (!std::isfinite(px[i])) return fail(BDRS_E_INVALID, "x has a non-finite entry at %zu", i);
  for (size_t i = 0; i < (size_t)n * dim; ++i)
    if (!std::isfinite(py[i])) return fail(BDRS_E_INVALID, "y has a non-finite entry at %zu", i);
  double sr = 0, sc = 0;
  for (int i = 0; i < m; ++i) {
    if (!(pr[i] > 0 && std::isfinite(pr[i]))) return fail(BDRS_E_INVALID, "r[%d] is not finite and > 0", i);
    sr += pr[i];
  }
  for (int j = 0; j < n; ++j) {
    if (!(pc[j] > 0 && std::isfinite(pc[j]))) return fail(BDRS_E_INVALID, "c[%d] is not finite and > 0", j);
    sc += pc[j];
  }
  if (std::fabs(sr - 1.0) > 1e-9) return fail(BDRS_E_INVALID, "r must sum to 1 (sum - 1 = %.3e)", sr - 1.0);
  if (std::fabs(sc - 1.0) > 1e-9) return fail(BDRS_E_INVALID, "c must sum to 1 (sum - 1 = %.3e)", sc - 1.0);
  img.m = m;
  img.n = n;
  img.dim = dim;
  // common origin: centre of the joint bounding box (keeps coordinates small)
  for (int d = 0; d < 3; ++d) img.origin[d] = 0.0;
  for (int d = 0; d < dim; ++d) {
    double lo = px[d], hi = px[d];
    for (int i = 0; i < m; ++i) lo = std::min(lo, (double)px[(size_t)i * dim + d]), hi = std::max(hi, (double)px[(size_t)i * dim + d]);
    for (int j = 0; j < n; ++j) lo = std::min(lo, (double)py[(size_t)j * dim + d]), hi = std::max(hi, (double)py[(size_t)j * dim + d]);
    img.origin[d] = (double)(float)(0.5 * (lo + hi));
  }
  build_side(px, pr, m, dim, img.origin, side_shape(m), img.R);
  build_side(py, pc, n, dim, img.origin, side_shape(n), img.C);
  return BDRS_OK;
}

bdrs_status create_from_image(const bdrs_params* p, const HostImage& img, bdrs_solver* out, int reserve_row,
                              int reserve_col) {
  *out = nullptr;
  const int m = p->m, n = p->n, dim = p->dim;
  if (img.m != m || img.n != n || img.dim != dim) return fail(BDRS_E_INVALID, "host image does not match the sizes");
  hipStream_t stream = (hipStream_t)p->stream;
  const Layout L = make_layout(m, n, dim, reserve_row, reserve_col, (p->flags & BDRS_F_KEEP_BEST_STATE) != 0);
  if (p->workspace_bytes < L.total)  // e.g. the tuning table changed since the workspace was sized
    return fail(BDRS_E_NOMEM, "workspace too small: %zu bytes given, %zu needed", p->workspace_bytes, L.total);
  bdrs_solver s = new bdrs_solver_();
  s->prm = *p;
  s->L = L;
  fill_ctx(s);
  for (int d = 0; d < 3; ++d) s->ctx.origin[d] = img.origin[d];
  const HostSide& R = img.R;
  const HostSide& C = img.C;

  const LaunchCtx& c = s->ctx;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
  };
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  chk(up(c.rows.abs, R.abs.data(), R.abs.size() * sizeof(float)));
  chk(up(c.rows.off, R.off.data(), R.off.size() * sizeof(float)));
  chk(up(c.rows.tile, R.tile.data(), R.tile.size() * sizeof(TileRec)));
  chk(up((void*)c.rows.geom, R.geom.data(), R.geom.size() * sizeof(TileGeom)));
  chk(up(c.rows.perm, R.perm.data(), R.perm.size() * sizeof(int)));
  chk(up(c.rows.iperm, R.iperm.data(), R.iperm.size() * sizeof(int)));
  chk(up(c.cols.iperm, C.iperm.data(), C.iperm.size() * sizeof(int)));
  chk(hipMemsetAsync(c.rows.hint, 0xff, sizeof(int) * (size_t)c.rows.np, stream));  // -1: no hint yet
  chk(hipMemsetAsync(c.cols.hint, 0xff, sizeof(int) * (size_t)c.cols.np, stream));
  chk(up(c.rows.marg, R.marg.data(), R.marg.size() * sizeof(double)));
  chk(up(c.rows.logmarg, R.logm.data(), R.logm.size() * sizeof(double)));
  chk(up(c.cols.abs, C.abs.data(), C.abs.size() * sizeof(float)));
  chk(up(c.cols.off, C.off.data(), C.off.size() * sizeof(float)));
  chk(up(c.cols.tile, C.tile.data(), C.tile.size() * sizeof(TileRec)));
  chk(up((void*)c.cols.geom, C.geom.data(), C.geom.size() * sizeof(TileGeom)));
  chk(up(c.cols.perm, C.perm.data(), C.perm.size() * sizeof(int)));
  chk(up(c.cols.marg, C.marg.data(), C.marg.size() * sizeof(double)));
  chk(up(c.cols.logmarg, C.logm.data(), C.logm.size() * sizeof(double)));
  Ctrl hc0{};
  hc0.k = 0;
  hc0.eta = p->eta;
  hc0.lam = p->lambda;
  hc0.scale = p->cost_scale;
  hc0.omega = p->omega;
  hc0.variant = p->flags & (BDRS_F_OLD_KERNEL | BDRS_F_NO_MOMENTUM | BDRS_F_DEBIASED);
  chk(up(c.ctrl, &hc0, sizeof hc0));
  // Algorithm 1 initialisation: log alpha^{-1} = log beta^{-1} = log beta^{-2} = 0
  chk(hipMemsetAsync(c.st.la, 0, sizeof(double) * c.rows.np, stream));
  chk(hipMemsetAsync(c.st.lah, 0, sizeof(double) * c.rows.np, stream));
  chk(hipMemsetAsync(c.st.lb1, 0, sizeof(double) * c.cols.np, stream));
  chk(hipMemsetAsync(c.st.lb2, 0, sizeof(double) * c.cols.np, stream));
  chk(hipMemsetAsync(c.st.lbh, 0, sizeof(double) * c.cols.np, stream));
  chk(hipMemsetAsync(c.st.lt[0], 0, sizeof(double) * c.cols.np, stream));
  chk(hipMemsetAsync(c.st.lt[1], 0, sizeof(double) * c.cols.np, stream));
  chk(hipMemsetAsync(c.cert_out, 0, sizeof(double) * kCertSlots, stream));
  if (e == hipSuccess) e = launch_prologue(c);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);  // the host image may go out of scope
  if (e != hipSuccess) {
    delete s;
    return fail(BDRS_E_DEVICE, "HIP error %s while initialising the workspace", hipGetErrorString(e));
  }
  *out = s;
  return BDRS_OK;
}

bdrs_status create_from_host(const bdrs_params* p, const float* px, const float* py, const double* pr,
                             const double* pc, bdrs_solver* out, int reserve_row, int reserve_col) {
  *out = nullptr;
  HostImage img;
  const bdrs_status st = prepare_image(p, px, py, pr, pc, img);
  if (st != BDRS_OK) return st;
  return create_from_image(p, img, out, reserve_row, reserve_col);
}

}  // namespace bdrs_host

extern "C" {

bdrs_status bdrs_step(bdrs_solver s, int32_t iters) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  if (iters < 0) return fail(BDRS_E_INVALID, "iters must be >= 0");
  if (iters == 0) return BDRS_OK;
  for (int32_t i = 0; i < iters; ++i) {
    bdrs_status st = enqueue_iteration(s, false, i);
    if (st != BDRS_OK) return st;
  }
  hipError_t e = launch_advance(s->ctx.ctrl, iters, s->ctx.stream);
  if (e != hipSuccess) return hip_status(e, "advance");
  s->k += iters;
  return BDRS_OK;
}

bdrs_status bdrs_certificate(bdrs_solver s, bdrs_cert* out) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  if (!out) return fail(BDRS_E_INVALID, "out is NULL");
  bdrs_status st = sync_k(s);
  if (st != BDRS_OK) return st;
  if (s->k < 1) return fail(BDRS_E_STATE, "no iteration has run yet");
  if ((st = enqueue_cert_only(s)) != BDRS_OK) return st;
  const LaunchCtx& c = s->ctx;
  hipError_t e;
  if ((e = launch_cert_reduce(c)) != hipSuccess) return hip_status(e, "cert reduce");
  const bool repair = (s->prm.flags & BDRS_F_REPAIR) != 0;
  if (repair && (st = enqueue_repair(s)) != BDRS_OK) return st;
  return read_cert(s, repair, out);
}

// One block of L iterations of Algorithm 1 ending with the fused certificate,
// the counter advance and the certificate reductions, captured once on a
// private stream and replayed on the solver's stream (every kernel reads the
// iteration counter from device memory, so one graph holds for all blocks).
bdrs_status launch_block_graph(bdrs_solver s, int L) {
  if (!s->blk_exec || s->blk_len != L) {
    if (s->blk_exec) {
      (void)hipGraphExecDestroy(s->blk_exec);
      s->blk_exec = nullptr;
      s->blk_len = 0;
    }
    if (!s->cap_stream) HIPCHK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    const hipStream_t user = s->ctx.stream;
    s->ctx.stream = s->cap_stream;
    hipGraph_t g = nullptr;
    bdrs_status st = BDRS_OK;
    hipError_t e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (int i = 0; i < L && st == BDRS_OK; ++i) st = enqueue_iteration(s, i == L - 1, i);
      if (st == BDRS_OK) e = launch_advance(s->ctx.ctrl, L, s->ctx.stream);
      if (st == BDRS_OK && e == hipSuccess) e = launch_cert_reduce(s->ctx);
      const hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
      if (e == hipSuccess) e = e2;
    }
    s->ctx.stream = user;
    if (e == hipSuccess && st == BDRS_OK) e = hipGraphInstantiate(&s->blk_exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (st != BDRS_OK) return st;
    if (e != hipSuccess) {
      s->blk_exec = nullptr;
      return hip_status(e, "block graph");
    }
    s->blk_len = L;
  }
  HIPCHK(hipGraphLaunch(s->blk_exec, s->ctx.stream));
  return BDRS_OK;
}

bdrs_status bdrs_solve(bdrs_solver s, double tau, int32_t tau_relative, int32_t max_iters, int32_t cert_every,
                       bdrs_cert* out) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  if (!(tau >= 0 && std::isfinite(tau))) return fail(BDRS_E_INVALID, "tau must be finite and >= 0");
  if (max_iters < 1) return fail(BDRS_E_INVALID, "max_iters must be >= 1");
  if (cert_every < 1) return fail(BDRS_E_INVALID, "cert_every must be >= 1");
  const bool repair = (s->prm.flags & BDRS_F_REPAIR) != 0;
  bdrs_cert ce{};
  bool have = false;
  bdrs_status st0 = sync_k(s);
  if (st0 != BDRS_OK) return st0;
  // the captured block needs the certificate fused into the last iteration
  // and no host-computed temperature (separate certificate sweep, repair)
  const bool graphs = !repair && !separate_cert(s) && !(s->prm.flags & BDRS_F_NO_GRAPH) && !s->prof;
  int pending = 0;  // iterations enqueued since the counter was last advanced
  for (int32_t i = 0; i < max_iters;) {
    const long long k = s->k + pending;
    bdrs_status st;
    if (graphs && pending == 0 && k % cert_every == 0 && max_iters - i >= cert_every) {
      if ((st = launch_block_graph(s, cert_every)) != BDRS_OK) return st;
      s->k += cert_every;
      i += cert_every;
      s->packed_rows = true;
    } else {
      const bool due = ((k + 1) % cert_every == 0) || (i == max_iters - 1);
      st = enqueue_iteration(s, due && !separate_cert(s), pending);
      if (st != BDRS_OK) return st;
      ++pending;
      ++i;
      if (!due) continue;
      hipError_t e;
      if ((e = launch_advance(s->ctx.ctrl, pending, s->ctx.stream)) != hipSuccess) return hip_status(e, "advance");
      s->k += pending;
      pending = 0;
      if (separate_cert(s) && (st = enqueue_cert_only(s)) != BDRS_OK) return st;
      if ((e = launch_cert_reduce(s->ctx)) != hipSuccess) return hip_status(e, "cert reduce");
      if (repair && (st = enqueue_repair(s)) != BDRS_OK) return st;
    }
    st = read_cert(s, repair, &ce);
    have = true;
    if (st != BDRS_OK) {
      if (out) *out = ce;
      return st;
    }
    const double target = tau_relative ? ce.rel_gap_best : (ce.U_best - ce.L_best);
    if (target <= tau) {
      if (out) *out = ce;
      return BDRS_OK;
    }
  }
  if (out && have) *out = ce;
  return BDRS_NOT_CONVERGED;
}

bdrs_status bdrs_get_state(bdrs_solver s, double* log_alpha, double* log_beta, double* log_beta_prev,
                           double* log_alpha_hat, double* log_beta_hat, double* log_beta_tilde, int64_t* iters_done) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  bdrs_status st = sync_k(s);
  if (st != BDRS_OK) return st;
  const LaunchCtx& c = s->ctx;
  hipError_t e = hipSuccess;
  auto sc = [&](const double* src, const SideDev& sd, double* dst) {
    if (dst && e == hipSuccess) e = launch_scatter(src, sd.perm, sd.count, dst, c.stream);
  };
  sc(c.st.la, c.rows, log_alpha);
  sc(c.st.lb1, c.cols, log_beta);
  sc(c.st.lb2, c.cols, log_beta_prev);
  sc(c.st.lah, c.rows, log_alpha_hat);
  sc(c.st.lbh, c.cols, log_beta_hat);
  // beta-tilde used by the last finished iteration k-1 sits in buffer (k-1) & 1
  sc(c.st.lt[(s->k + 1) & 1], c.cols, log_beta_tilde);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e != hipSuccess) return hip_status(e, "get_state");
  if (iters_done) *iters_done = s->k;
  return BDRS_OK;
}

bdrs_status bdrs_set_state(bdrs_solver s, const double* log_alpha, const double* log_beta,
                           const double* log_beta_prev, const double* log_alpha_hat, const double* log_beta_hat,
                           const double* log_beta_tilde, int64_t iters_done) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  if (!log_alpha || !log_beta || !log_beta_prev)
    return fail(BDRS_E_INVALID, "log_alpha, log_beta and log_beta_prev are required");
  if (iters_done < 0) return fail(BDRS_E_INVALID, "iters_done must be >= 0");
  const LaunchCtx& c = s->ctx;
  hipError_t e = hipSuccess;
  auto ga = [&](const double* src, const SideDev& sd, double* dst) {
    if (src && e == hipSuccess) e = launch_gather(src, sd.perm, sd.np, dst, c.stream);
  };
  ga(log_alpha, c.rows, c.st.la);
  ga(log_beta, c.cols, c.st.lb1);
  ga(log_beta_prev, c.cols, c.st.lb2);
  ga(log_alpha_hat, c.rows, c.st.lah);
  ga(log_beta_hat, c.cols, c.st.lbh);
  ga(log_beta_tilde, c.cols, c.st.lt[(iters_done + 1) & 1]);
  if (e != hipSuccess) return hip_status(e, "set_state");
  long long k = iters_done;
  HIPCHK(hipMemcpyAsync(&c.ctrl->k, &k, sizeof k, hipMemcpyHostToDevice, c.stream));
  s->k = k;
  s->U_best = INFINITY;
  s->L_best = -INFINITY;
  s->kU = s->kL = -1;
  s->packed_rows = false;
  bdrs_status st = BDRS_OK;
  if (log_alpha_hat) st = repack(s);
  else {
    hipError_t e2 = launch_prologue(c);
    if (e2 != hipSuccess) st = hip_status(e2, "prologue");
  }
  if (st != BDRS_OK) return st;
  HIPCHK(hipStreamSynchronize(c.stream));
  return BDRS_OK;
}

bdrs_status bdrs_lse(bdrs_solver s, int32_t transpose, double eps, const double* w, double* out) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  if (!w || !out) return fail(BDRS_E_INVALID, "w and out are required");
  if (!(eps > 0 && std::isfinite(eps))) return fail(BDRS_E_INVALID, "eps must be finite and > 0");
  const LaunchCtx& c = s->ctx;
  const bool tr = transpose != 0;
  const int splits = tr ? s->L.splits_col : s->L.splits_row;
  hipError_t e;
  if ((e = launch_pack(c, tr, w, eps)) != hipSuccess) return hip_status(e, "pack");
  bdrs_status st = sync_k(s);
  if (st != BDRS_OK) return st;
  if ((e = sweep(s, tr, false, splits, eps)) != hipSuccess) return hip_status(e, "sweep");
  if ((e = launch_finish(c, tr, kFinishLse, splits, eps, out, 0)) != hipSuccess) return hip_status(e, "finish");
  s->packed_rows = false;
  return repack(s);
}

bdrs_status bdrs_plan(bdrs_solver s, double* bary, double* row_marg, double* col_marg, bdrs_plan_stats* out) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  bdrs_status st = sync_k(s);
  if (st != BDRS_OK) return st;
  if (s->k < 1) return fail(BDRS_E_STATE, "the state plan needs at least one finished iteration");
  const LaunchCtx& c = s->ctx;
  // X^k = diag(alpha^{k-1}) K^{.lambda k} diag(beta^{k-1}): kernel temperature eta / (lambda k)
  const double eps = s->prm.eta / (s->prm.lambda * (double)s->k);
  hipError_t e;
  if ((e = launch_pack_state(c, false, eps)) != hipSuccess) return hip_status(e, "pack beta");
  if ((e = launch_sweep_bary(c, s->L.splits_row, eps)) != hipSuccess) return hip_status(e, "row sweep");
  if ((e = launch_finish(c, false, kFinishPlanRow, s->L.splits_row, eps, bary, 0)) != hipSuccess)
    return hip_status(e, "row finish");
  if ((e = launch_pack_state(c, true, eps)) != hipSuccess) return hip_status(e, "pack alpha");
  if ((e = sweep(s, true, false, s->L.splits_col, eps)) != hipSuccess) return hip_status(e, "column sweep");
  if ((e = launch_finish(c, true, kFinishPlanCol, s->L.splits_col, eps, nullptr, 0)) != hipSuccess)
    return hip_status(e, "column finish");
  if ((e = launch_plan_stats(c)) != hipSuccess) return hip_status(e, "statistics");
  // tile order -> caller order
  if (row_marg && (e = launch_scatter(c.plan_row, c.rows.perm, c.rows.count, row_marg, c.stream)) != hipSuccess)
    return hip_status(e, "row scatter");
  if (col_marg && (e = launch_scatter(c.plan_col, c.cols.perm, c.cols.count, col_marg, c.stream)) != hipSuccess)
    return hip_status(e, "column scatter");
  double h[kCertSlots];
  HIPCHK(hipMemcpyAsync(h, c.plan_stats, sizeof(double) * 8, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  if (out) {
    out->k = s->k;
    out->eps = eps;
    out->row_l1 = h[0];
    out->row_max_abs = h[1];
    out->row_max_rel = h[2];
    out->col_l1 = h[3];
    out->col_max_abs = h[4];
    out->col_max_rel = h[5];
    out->mass = h[6];
  }
  s->packed_rows = false;
  return repack(s);
}

// Two-sided rounding of the state plan X = diag(alpha) K diag(beta) at eps
// (Altschuler, Weed and Rigollet 2017, Algorithm 2) in three sweeps: log x in
// plan_row, log y in plan_col, e_r in plan_aux, e_c in mu, <C, G> and
// ||e_r||_1 in plan_stats[8..11].  The rows are left packed with other weights.
bdrs_status enqueue_round(bdrs_solver s, double eps) {
  const LaunchCtx& c = s->ctx;
  hipError_t e;
  // 1: row sums of X and x = min(1, r / X 1)
  if ((e = launch_pack_state(c, false, eps)) != hipSuccess) return hip_status(e, "pack beta");
  if ((e = sweep(s, false, false, s->L.splits_row, eps)) != hipSuccess) return hip_status(e, "row sweep");
  if ((e = launch_finish(c, false, kFinishRound1, s->L.splits_row, eps, nullptr, 0)) != hipSuccess)
    return hip_status(e, "row finish");
  // 2: column sums of diag(x) X and y = min(1, c / .)
  if ((e = launch_pack_state(c, true, eps, true)) != hipSuccess) return hip_status(e, "pack alpha x");
  if ((e = sweep(s, true, false, s->L.splits_col, eps)) != hipSuccess) return hip_status(e, "column sweep");
  if ((e = launch_finish(c, true, kFinishRound2, s->L.splits_col, eps, nullptr, 0)) != hipSuccess)
    return hip_status(e, "column finish");
  // 3: row sums and cost of diag(x) X diag(y)
  if ((e = launch_pack_state(c, false, eps, true)) != hipSuccess) return hip_status(e, "pack beta y");
  if ((e = sweep(s, false, true, s->L.splits_row, eps)) != hipSuccess) return hip_status(e, "cost sweep");
  if ((e = launch_finish(c, false, kFinishRound3, s->L.splits_row, eps, nullptr, 0)) != hipSuccess)
    return hip_status(e, "cost finish");
  if ((e = launch_round_reduce(c)) != hipSuccess) return hip_status(e, "reduce");
  s->packed_rows = false;
  return BDRS_OK;
}

bdrs_status bdrs_round(bdrs_solver s, bdrs_round_stats* out) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  if (!out) return fail(BDRS_E_INVALID, "out is NULL");
  bdrs_status st = sync_k(s);
  if (st != BDRS_OK) return st;
  if (s->k < 1) return fail(BDRS_E_STATE, "rounding needs at least one finished iteration");
  const double eps = s->prm.eta / (s->prm.lambda * (double)s->k);  // the state plan's kernel
  if ((st = enqueue_round(s, eps)) != BDRS_OK) return st;
  const LaunchCtx& c = s->ctx;
  double h[4];
  HIPCHK(hipMemcpyAsync(h, c.plan_stats + 8, sizeof h, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  out->k = s->k;
  out->eps = eps;
  out->cost = h[0];
  out->cost_clipped = h[1];
  out->mass_moved = h[2];
  if (!std::isfinite(h[0])) return fail(BDRS_E_NUMERIC, "non-finite rounded cost");
  return repack(s);
}

bdrs_status bdrs_export_plan(bdrs_solver s, int32_t kind, double* log_u, double* log_v, double* a, double* b,
                             bdrs_plan_export* out) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  if (kind != BDRS_PLAN_ROUNDED && kind != BDRS_PLAN_REPAIRED) return fail(BDRS_E_INVALID, "unknown plan kind %d", kind);
  bdrs_status st = sync_k(s);
  if (st != BDRS_OK) return st;
  if (s->k < 1) return fail(BDRS_E_STATE, "a plan needs at least one finished iteration");
  const LaunchCtx& c = s->ctx;
  hipError_t e;
  double h[kCertSlots];
  bdrs_plan_export info{};
  info.kind = kind;
  info.k = s->k;
  info.cost_scale = s->prm.cost_scale;
  if (kind == BDRS_PLAN_ROUNDED) {
    const double eps = s->prm.eta / (s->prm.lambda * (double)s->k);
    if ((st = enqueue_round(s, eps)) != BDRS_OK) return st;
    if ((e = launch_export_factors(c, false, nullptr, log_u, log_v, a, b)) != hipSuccess)
      return hip_status(e, "export factors");
    HIPCHK(hipMemcpyAsync(h, c.plan_stats + 8, 4 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    info.eps = eps;
    info.cost = h[0];
    info.mass = h[2];
    if ((st = repack(s)) != BDRS_OK) return st;
  } else {
    // the certificate's column statistics and the repair of the last finished iteration
    if ((st = enqueue_cert_only(s)) != BDRS_OK) return st;
    if ((e = launch_cert_reduce(c)) != hipSuccess) return hip_status(e, "cert reduce");
    if ((st = enqueue_repair(s)) != BDRS_OK) return st;
    if ((e = launch_export_factors(c, true, c.st.lt[(s->k - 1) & 1], log_u, log_v, a, b)) != hipSuccess)
      return hip_status(e, "export factors");
    HIPCHK(hipMemcpyAsync(h, c.cert_out, sizeof h, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    info.eps = h[1];
    info.cost = h[8];
    info.mass = h[4];
  }
  if (out) *out = info;
  if (!std::isfinite(info.cost)) return fail(BDRS_E_NUMERIC, "non-finite plan cost");
  return BDRS_OK;
}

bdrs_status bdrs_plan_entries(bdrs_solver s, const double* log_u, const double* log_v, const double* a,
                              const double* b, double eps, int64_t row_begin, int64_t row_end, double* out) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  if (!log_u || !log_v || (!out && row_end > row_begin))
    return fail(BDRS_E_INVALID, "log_u, log_v and out must not be NULL");
  if ((a == nullptr) != (b == nullptr)) return fail(BDRS_E_INVALID, "a and b must both be given or both be NULL");
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(BDRS_E_INVALID, "eps must be positive and finite");
  const LaunchCtx& c = s->ctx;
  if (row_begin < 0 || row_end < row_begin || row_end > c.rows.count)
    return fail(BDRS_E_INVALID, "row range [%lld, %lld) outside [0, %d)", (long long)row_begin, (long long)row_end,
                c.rows.count);
  if (c.cols.count > 65535 * kBlock) return fail(BDRS_E_INVALID, "dense entries need n <= %d", 65535 * kBlock);
  const hipError_t e = launch_plan_entries(c, log_u, log_v, a, b, s->prm.cost_scale / eps, row_begin,
                                           row_end - row_begin, out);
  if (e != hipSuccess) return hip_status(e, "plan entries");
  HIPCHK(hipStreamSynchronize(c.stream));
  return BDRS_OK;
}

bdrs_status bdrs_get_hints(bdrs_solver s, int32_t* row_hint, int32_t* col_hint) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  const LaunchCtx& c = s->ctx;
  hipError_t e = hipSuccess;
  if (row_hint) e = launch_hints_out(c.rows.hint, c.rows.perm, c.cols.perm, c.rows.count, row_hint, c.stream);
  if (e == hipSuccess && col_hint)
    e = launch_hints_out(c.cols.hint, c.cols.perm, c.rows.perm, c.cols.count, col_hint, c.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  return e == hipSuccess ? BDRS_OK : hip_status(e, "get_hints");
}

bdrs_status bdrs_set_hints(bdrs_solver s, const int32_t* row_hint, const int32_t* col_hint) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  const LaunchCtx& c = s->ctx;
  hipError_t e = hipSuccess;
  if (row_hint) e = launch_hints_in(row_hint, c.rows.perm, c.cols.iperm, c.cols.count, c.rows.np, c.rows.hint, c.stream);
  if (e == hipSuccess && col_hint)
    e = launch_hints_in(col_hint, c.cols.perm, c.rows.iperm, c.rows.count, c.cols.np, c.cols.hint, c.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  return e == hipSuccess ? BDRS_OK : hip_status(e, "set_hints");
}

bdrs_status bdrs_profile(bdrs_solver s, int32_t enable) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  HIPCHK(hipStreamSynchronize(s->ctx.stream));
  s->prof = enable != 0;
  if (s->prof) {
    s->ev_used = 0;
    s->prof_entries = 0.0;
    s->prof_sweeps = 0;
    char* base = (char*)s->prm.workspace;
    HIPCHK(hipMemsetAsync(base + s->L.tile_total, 0, sizeof(unsigned long long), s->ctx.stream));
    HIPCHK(hipStreamSynchronize(s->ctx.stream));
  }
  return BDRS_OK;
}

bdrs_status bdrs_profile_evaluated(bdrs_solver s, double* entries) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  if (!entries) return fail(BDRS_E_INVALID, "entries is NULL");
  unsigned long long tiles = 0;
  HIPCHK(hipMemcpyAsync(&tiles, (char*)s->prm.workspace + s->L.tile_total, sizeof tiles, hipMemcpyDeviceToHost,
                        s->ctx.stream));
  HIPCHK(hipStreamSynchronize(s->ctx.stream));
  *entries = (double)tiles * (double)kTile * (double)kTile;  // (64 outputs) x (64 inputs) per count
  return BDRS_OK;
}

bdrs_status bdrs_profile_read(bdrs_solver s, int64_t* sweeps, double* ms, double* entries) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  HIPCHK(hipStreamSynchronize(s->ctx.stream));
  double tot = 0.0;
  for (size_t i = 0; i + 1 < s->ev_used; i += 2) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, s->ev_pool[i], s->ev_pool[i + 1]));
    tot += t;
  }
  if (sweeps) *sweeps = s->prof_sweeps;
  if (ms) *ms = tot;
  if (entries) *entries = s->prof_entries;
  return BDRS_OK;
}

bdrs_status bdrs_restore_best(bdrs_solver s, int64_t* iters_done) {
  if (!s) return fail(BDRS_E_INVALID, "solver is NULL");
  if (!s->L.keep_best) return fail(BDRS_E_INVALID, "the solver was created without BDRS_F_KEEP_BEST_STATE");
  if (s->best_k < 0) return fail(BDRS_E_STATE, "no certificate yet: no state retained");
  const LaunchCtx& c = s->ctx;
  HIPCHK(copy_best(s, false));
  long long k = s->best_k;
  HIPCHK(hipMemcpyAsync(&c.ctrl->k, &k, sizeof k, hipMemcpyHostToDevice, c.stream));
  s->k = k;
  s->packed_rows = false;
  const bdrs_status st = repack(s);
  if (st != BDRS_OK) return st;
  HIPCHK(hipStreamSynchronize(c.stream));
  if (iters_done) *iters_done = k;
  return BDRS_OK;
}

bdrs_status bdrs_destroy(bdrs_solver s) {
  if (!s) return BDRS_OK;
  hipError_t e = hipStreamSynchronize(s->ctx.stream);
  // teardown: nothing to report
  for (hipEvent_t ev : s->ev_pool) (void)hipEventDestroy(ev);
  if (s->blk_exec) (void)hipGraphExecDestroy(s->blk_exec);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
  if (e != hipSuccess) return hip_status(e, "destroy");
  return BDRS_OK;
}

}  // extern "C"
