/*
 * The C ABI of include/bdrs.h used from plain C, without Python: two grid
 * histograms (side x side pixels, each a Gaussian bump on a 1e-6 floor,
 * normalised), the squared Euclidean cost of the unit grid halved (integer
 * coordinates with cost scale 1 / (2 (side - 1)^2)), solved with Dual BDRS
 * to a certified relative gap, then the state plan rounded onto Pi(r, c),
 * and the repaired plan of the last iteration exported (factors) and written
 * out densely, whose row and column sums are checked against r and c.
 *
 * usage: solve_grid [side=64] [eta=0.1] [lambda=1] [tau=0.01]
 * prints one line "k L_best U_best rel_gap_best rounded_cost seconds
 * repaired_cost max_marginal_error" and exits 0 when L_best <= rounded_cost,
 * L_best <= repaired_cost and the dense repaired plan's marginals match r
 * and c to 1e-4 relative.
 */
#define _POSIX_C_SOURCE 199309L
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <time.h>

#include "bdrs.h"

#define HIP_OK(call)                                                            \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));                \
      return 2;                                                                 \
    }                                                                           \
  } while (0)

#define BDRS_OK(call)                                                           \
  do {                                                                          \
    bdrs_status s_ = (call);                                                    \
    if (s_ < 0) {                                                               \
      fprintf(stderr, "%s: status %d: %s\n", #call, (int)s_, bdrs_last_error()); \
      return 3;                                                                 \
    }                                                                           \
  } while (0)

static void bump(double *h, int side, double cx, double cy, double sigma) {
  double sum = 0.0;
  for (int i = 0; i < side; ++i)
    for (int j = 0; j < side; ++j) {
      const double u = (double)i / (side - 1) - cx, v = (double)j / (side - 1) - cy;
      h[i * side + j] = exp(-(u * u + v * v) / (2.0 * sigma * sigma));
      sum += h[i * side + j];
    }
  double sum2 = 0.0;
  for (int k = 0; k < side * side; ++k) {
    h[k] = h[k] / sum + 1e-6;
    sum2 += h[k];
  }
  for (int k = 0; k < side * side; ++k) h[k] /= sum2;
}

int main(int argc, char **argv) {
  const int side = argc > 1 ? atoi(argv[1]) : 64;
  const double eta = argc > 2 ? atof(argv[2]) : 0.1;
  const double lam = argc > 3 ? atof(argv[3]) : 1.0;
  const double tau = argc > 4 ? atof(argv[4]) : 0.01;
  if (side < 2) {
    fprintf(stderr, "side must be >= 2\n");
    return 1;
  }
  const int n = side * side;
  float *pts = malloc(sizeof(float) * 2 * n);
  double *r = malloc(sizeof(double) * n), *c = malloc(sizeof(double) * n);
  for (int i = 0; i < side; ++i)
    for (int j = 0; j < side; ++j) {
      pts[2 * (i * side + j)] = (float)i;
      pts[2 * (i * side + j) + 1] = (float)j;
    }
  bump(r, side, 0.3, 0.35, 0.15);
  bump(c, side, 0.65, 0.6, 0.2);

  bdrs_params p = {0};
  p.m = n;
  p.n = n;
  p.dim = 2;
  p.cost_scale = 1.0 / (2.0 * (side - 1) * (side - 1));
  p.eta = eta;
  p.lambda = lam;
  p.omega = 1.0;
  size_t ws_bytes = 0;
  BDRS_OK(bdrs_workspace_size(&p, &ws_bytes));

  void *dx, *dy, *dr, *dc, *ws;
  HIP_OK(hipMalloc(&dx, sizeof(float) * 2 * n));
  HIP_OK(hipMalloc(&dy, sizeof(float) * 2 * n));
  HIP_OK(hipMalloc(&dr, sizeof(double) * n));
  HIP_OK(hipMalloc(&dc, sizeof(double) * n));
  HIP_OK(hipMalloc(&ws, ws_bytes));  /* hipMalloc returns 256-byte aligned memory */
  HIP_OK(hipMemcpy(dx, pts, sizeof(float) * 2 * n, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dy, pts, sizeof(float) * 2 * n, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dr, r, sizeof(double) * n, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dc, c, sizeof(double) * n, hipMemcpyHostToDevice));
  p.x = dx;
  p.y = dy;
  p.r = dr;
  p.c = dc;
  p.workspace = ws;
  p.workspace_bytes = ws_bytes;
  p.stream = NULL;

  bdrs_solver s = NULL;
  BDRS_OK(bdrs_create(&p, &s));
  bdrs_cert ce;
  struct timespec t0, t1;
  clock_gettime(CLOCK_MONOTONIC, &t0);
  const bdrs_status st = bdrs_solve(s, tau, 1, 40000, 50, &ce);
  clock_gettime(CLOCK_MONOTONIC, &t1);
  BDRS_OK(st);
  bdrs_round_stats rs;
  BDRS_OK(bdrs_round(s, &rs));
  const double secs = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);

  /* the repaired plan: factors on the device, then its dense rows in strips */
  void *du, *dv, *da, *db, *dp;
  HIP_OK(hipMalloc(&du, sizeof(double) * n));
  HIP_OK(hipMalloc(&dv, sizeof(double) * n));
  HIP_OK(hipMalloc(&da, sizeof(double) * n));
  HIP_OK(hipMalloc(&db, sizeof(double) * n));
  bdrs_plan_export pe;
  BDRS_OK(bdrs_export_plan(s, BDRS_PLAN_REPAIRED, du, dv, da, db, &pe));
  const int strip = 64;
  HIP_OK(hipMalloc(&dp, sizeof(double) * (size_t)strip * n));
  double *hp = malloc(sizeof(double) * (size_t)strip * n), *col = calloc((size_t)n, sizeof(double));
  double err = 0.0;
  for (int i0 = 0; i0 < n; i0 += strip) {
    const int i1 = i0 + strip < n ? i0 + strip : n;
    BDRS_OK(bdrs_plan_entries(s, du, dv, da, db, pe.eps, i0, i1, dp));
    HIP_OK(hipMemcpy(hp, dp, sizeof(double) * (size_t)(i1 - i0) * n, hipMemcpyDeviceToHost));
    for (int i = i0; i < i1; ++i) {
      double row = 0.0;
      for (int j = 0; j < n; ++j) {
        row += hp[(size_t)(i - i0) * n + j];
        col[j] += hp[(size_t)(i - i0) * n + j];
      }
      err = fmax(err, fabs(row - r[i]) / r[i]);
    }
  }
  for (int j = 0; j < n; ++j) err = fmax(err, fabs(col[j] - c[j]) / c[j]);
  printf("%lld %.12g %.12g %.6g %.12g %.4f %.12g %.3g\n", (long long)ce.k, ce.L_best, ce.U_best, ce.rel_gap_best,
         rs.cost, secs, pe.cost, err);
  HIP_OK(hipFree(dp));
  HIP_OK(hipFree(db));
  HIP_OK(hipFree(da));
  HIP_OK(hipFree(dv));
  HIP_OK(hipFree(du));
  free(hp);
  free(col);
  BDRS_OK(bdrs_destroy(s));
  HIP_OK(hipFree(ws));
  HIP_OK(hipFree(dc));
  HIP_OK(hipFree(dr));
  HIP_OK(hipFree(dy));
  HIP_OK(hipFree(dx));
  free(pts);
  free(r);
  free(c);
  const int ok = st == BDRS_OK && ce.L_best <= rs.cost * (1.0 + 1e-9) && ce.L_best <= pe.cost * (1.0 + 1e-9) &&
                 err <= 1e-4;
  return ok ? 0 : 4;
}
