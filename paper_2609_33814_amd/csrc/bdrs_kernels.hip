// gfx950 kernels of the Dual O-BDRS hot path.
//
// Sweep (the reduction of Algorithm 1's row and column updates, and of
// Algorithm 2's column pass).  For every output point p of one side and the
// input points q of the other side it evaluates, in base 2,
//     LSE2_p = log2 sum_q 2^{ w2_q - kappa2 ||P_p - Q_q||^2 },
//     kappa2 = log2(e) * s / eps,   w2 = log2(e) * w,
// which is LSE_q(w_q - C_pq / eps) / ln 2.  The cost is never stored: inputs
// are grouped in tiles of 64 spatially close points with centre Qc, offsets
// b_q = Q_q - Qc, and with a = P_p - Qc and the plane fit
// w2_q ~ alpha + gamma . b_q of the tile's weights the exponent expands
// exactly as
//     w2_q - kappa2 |a - b_q|^2 = base + B . b_q + A_q,
//     base = alpha - kappa2 |a|^2,  B = gamma + 2 kappa2 a,
//     A_q = w2_q - alpha - gamma . b_q - kappa2 |b_q|^2   (written by the producing epilogue),
// i.e. d FMAs and one add per entry, then one v_exp_f32 and one add.
//
// Precision split.  The weights w grow like g / eps as the temperature falls,
// so float32 values of that size would carry absolute errors u |g| / eps.  The
// inner loop therefore only sees small numbers: A_q is the weight's residual
// from its tile's plane minus the tile-local quadratic (float32), B is formed
// in float64 before it is rounded, and the large per-(output, tile) part base
// and the lane's running shift M are kept in float64.  The summand is
// 2^{cm + B . b_q + A_q} with cm = base - M (float32).  For the entries that
// dominate an output's sum B is the exponent's slope across the tile near its
// maximum, so every float32 operand is of the order of kappa2 r^2 (r the tile
// radius) rather than of the weights' variation across the tile, which at low
// temperature is 2 kappa2 |a| r, the transport distance |a| times larger.
//
// Stability without a per-entry max: the per-(output, tile) upper bound
//     UB = base + sum_d |2 kappa2 a_d| rad_d  >=  max_q exponent
// is compared with M.  Only when UB > M + 64 does the lane take the exact
// maximum of the tile first (and rescale its sum), so every summed term is at
// most 2^64 and M never exceeds the true maximum (no underflow of the leading
// terms).  Lanes of a wave hold 64 consecutive outputs in tile order, i.e.
// neighbouring points, so they agree on which tiles need the exact maximum.
//
// Each (block of 256 outputs, split of the input tiles) writes a partial
// (M, S[, N]); the finish kernels merge the splits in float64 and run the
// epilogue of Algorithm 1 (overrelaxation, momentum, packing of the next
// sweep's weights) or of Algorithm 2 (column mean costs and masses).
#include "bdrs_internal.h"

#include <hip/hip_ext.h>

#include <math.h>

#include <algorithm>

namespace bdrs {

namespace {

constexpr double kLog2eD = 1.4426950408889634074;
constexpr double kLn2D = 0.69314718055994530942;
// Exact-max gate: a tile whose bound exceeds the running shift by more than
// this takes its exact maximum first, so no summed term exceeds 2^64.
constexpr float kThresh = 64.0f;

// Skip gate of a sweep over n inputs: a tile whose bound lies more than
// T = 30 + ceil(log2 n) (at most 64) below an output's running shift M is
// skipped.  Every output's sum is at least 2^M (the term that set M is
// summed), and the skipped terms add at most n 2^{M-T} <= 2^{M-30}: 1/64 of
// float32's half-ulp, below the rounding of the float32 sum itself.
__device__ __forceinline__ double skip_threshold(int n) {
  return fmin(64.0, 30.0 + ceil(log2((double)max(n, 1))));
}

template <typename CtrlPtr>
__device__ __forceinline__ double eps_of(CtrlPtr c, double eps_arg, int kshift) {
  if (eps_arg > 0.0) return eps_arg;
  return c->eta / (c->lam * (double)(c->k + kshift) + 1.0);  // eta_k = eta / (lambda k + 1)
}

// Temperature of the row update: eta_k, or eta / k for the old kernel K^{.k}.
template <typename CtrlPtr>
__device__ __forceinline__ double eps_row_of(CtrlPtr c, double eps_arg, int kshift) {
  if (eps_arg > 0.0) return eps_arg;
  if (c->variant & kVarOldKernel) {
    const long long k = c->k + kshift;
    return k >= 1 ? c->eta / (double)k : c->eta * kFarTemperature;
  }
  return eps_of(c, -1.0, kshift);
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Wavefront all-reductions of a double with DPP lane moves inside each row of
// 16 lanes (swap neighbours, swap pairs, mirror halves, mirror the row) and
// four readlanes across the rows; every lane receives the result.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

constexpr int kDppXor1 = 0xB1;        // quad_perm(1, 0, 3, 2)
constexpr int kDppXor2 = 0x4E;        // quad_perm(2, 3, 0, 1)
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within each half row
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i within each row

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<kDppXor1>(v);
  v += dpp_move<kDppXor2>(v);
  v += dpp_move<kDppHalfMirror>(v);
  v += dpp_move<kDppMirror>(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// N independent sums at once (their lane moves interleave).
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<kDppXor1>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<kDppXor2>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<kDppHalfMirror>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_move<kDppMirror>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i)
    v[i] = (read_lane(v[i], 0) + read_lane(v[i], 16)) + (read_lane(v[i], 32) + read_lane(v[i], 48));
}

__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_move<kDppXor1>(v));
  v = fmax(v, dpp_move<kDppXor2>(v));
  v = fmax(v, dpp_move<kDppHalfMirror>(v));
  v = fmax(v, dpp_move<kDppMirror>(v));
  return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}

// ---------------------------------------------------------------------------
// Sweep
// ---------------------------------------------------------------------------
// Global-address-space views: the tile data is read through these so that
// uniform reads compile to scalar loads also when the pointers come from a
// descriptor in memory (batched launches), not only from kernel arguments.
typedef __attribute__((address_space(1))) const float gfloat;
typedef __attribute__((address_space(1))) const double gdouble;
typedef __attribute__((address_space(1))) const Ctrl gctrl;

typedef __attribute__((address_space(1))) const TileRec gtile;

// Points of a tile per group: the tile data of one group (8 D offsets into
// scalar registers, 8 weights into vector registers by broadcast loads) is
// requested while the previous group is being computed.
constexpr int kGroup = 8;

// The fields of a tile record the sweep uses (dimensions < D).
template <int D>
struct TileVals {
  double amax, alpha;
  float ctr[D], rad[D], gam[D], rho;
};

template <int D>
__device__ __forceinline__ TileVals<D> load_tile(gtile* __restrict__ rec) {
  gdouble* dp = (gdouble*)rec;
  gfloat* fp = (gfloat*)rec;
  TileVals<D> v;
  v.amax = dp[0];
  v.alpha = dp[1];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    v.ctr[d] = fp[4 + d];
    v.rad[d] = fp[7 + d];
    v.gam[d] = fp[10 + d];
  }
  v.rho = fp[13];
  return v;
}

template <int D>
struct Group {
  float b[D][kGroup];
  float a[kGroup];
};

// Group g of a tile whose offsets start at offs_t ([D][64]) and weights at a_t.
template <int D>
__device__ __forceinline__ Group<D> load_group(gfloat* __restrict__ offs_t, gfloat* __restrict__ a_t, int g) {
  Group<D> r;
  gfloat* offs = offs_t + g * kGroup;
  gfloat* aq = a_t + g * kGroup;
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int u = 0; u < kGroup; ++u) r.b[d][u] = offs[d * kTile + u];
#pragma unroll
  for (int u = 0; u < kGroup; ++u) r.a[u] = aq[u];
  return r;
}

// One block of kSweepBlock outputs (bx) against one split of the input tiles
// (every nsplit-th tile).  Per chunk of up to 64 tiles a coarse test against
// the wavefront's output box picks the candidate tiles; per candidate the lane
// bounds its own exponents and the wavefront skips the tile when no lane can
// see it, else every lane evaluates z_q = cm + B . b_q + A_q and accumulates
// exp2(z_q) (and, for the certificate, the cost-weighted sum).  The next group
// of 8 points (after a tile's last group, the next candidate's first) is
// requested before the current group is computed, so the loads overlap the
// arithmetic.
template <int D, int MODE>
__device__ __forceinline__ void sweep_block(
    gfloat* __restrict__ out_abs, int np_out,
    gfloat* __restrict__ in_off, gfloat* __restrict__ in_A, gtile* __restrict__ in_tile,
    int ntiles_in, int count_in, int nsplit, const int* __restrict__ hint,
    void* __restrict__ part, double* __restrict__ part_ref, gctrl* __restrict__ ctrl, double eps_arg, int kofs,
    int bx, int split, bool row_sweep, unsigned* __restrict__ tile_count, int slot) {
  constexpr bool CERT = MODE == kSweepCert;
  constexpr bool BARY = MODE == kSweepBary;
  const int p = bx * kSweepBlock + threadIdx.x;
  // Split `split` of nsplit takes every nsplit-th input tile (split, split +
  // nsplit, ...), so that each split samples the whole input cloud: late in a
  // solve only the tiles near an output block matter, and they spread over
  // all splits instead of crowding into one wavefront's work.  Local index i
  // is tile split + i nsplit; nt tiles in all.
  const int nt = split < ntiles_in ? (ntiles_in - 1 - split) / nsplit + 1 : 0;
  // the output point and its hint first: their loads do not wait for the
  // temperature, whose control-block reads sit behind branches
  float P[D];
#pragma unroll
  for (int d = 0; d < D; ++d) P[d] = out_abs[(size_t)d * np_out + p];
  const int j_hint = hint[p];
  const double eps = row_sweep ? eps_row_of(ctrl, eps_arg, kofs) : eps_of(ctrl, eps_arg, kofs);
  const double kap2d = kLog2eD * ctrl->scale / eps;
  const double kap2x2d = 2.0 * kap2d;
  const float kap2f = (float)kap2d;
  const float inv2kap = (float)(0.5 / kap2d);

  // The wavefront's output box (all lanes, padding included: a larger box
  // only loosens the coarse bound below) and the coarse bound of the first
  // chunk of tiles, computed before the warm start so that their loads overlap
  // its own.
  const int lane0 = (int)__builtin_amdgcn_mbcnt_lo(0u, 0u);
  const int lane = (int)(threadIdx.x & (kTile - 1));
  float blo[D], bhi[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    blo[d] = (float)(-wave_max(-(double)P[d]));
    bhi[d] = (float)wave_max((double)P[d]);
  }
  // Coarse test of up to 64 tiles at once, lane l taking tile c0 + l: an
  // upper bound of the exponents of the tile's points for every output of the
  // wavefront, alpha + sum_d |gamma_d| r_d + rho - kappa2 dist^2(output box,
  // tile box), to be compared with the smallest running maximum of the
  // wavefront.  It bounds each lane's own bound from above, so a tile it
  // rejects would be skipped by the per-lane test too.  Local indices c0 ...
  // c1-1; the tile index is clamped to a valid tile (also for an empty split).
  auto coarse = [&](int c0, int c1) -> double {
    const int il = max(min(c0 + lane, c1 - 1), 0);
    gtile* rec = in_tile + min(split + il * nsplit, ntiles_in - 1);
    gfloat* fp = (gfloat*)rec;
    const double alpha = ((gdouble*)rec)[1];
    float w = fp[13], g2 = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const float ctr = fp[4 + d], rad = fp[7 + d], gam = fp[10 + d];
      w = fmaf(fabsf(gam), rad, w);
      // gap between the boxes, shrunk by a relative 1e-5 against rounding
      const float gap = fmaxf(0.0f, fmaxf((ctr - rad) - bhi[d], blo[d] - (ctr + rad))) * 0.99999f;
      g2 = fmaf(gap, gap, g2);
    }
    return alpha + (double)fmaf(-kap2f, g2, w);
  };
  double cub = coarse(0, min(kTile, nt));

  // Warm start: the exact exponent of one remembered input point is a lower
  // bound of the output's maximum over all inputs, so it is a valid shift for
  // every split (a split whose terms all lie far below it adds ~nothing); it
  // spares the exact-max pass on the first tile of each split.  Its loads are
  // issued unconditionally at a clamped, valid index and the result is masked
  // afterwards: loads under a branch would wait for their data one by one.
  double M = -INFINITY;
  int J = -1;
  {
    const int j = j_hint;
    const int jc = min(max(j, 0), count_in - 1);
    const int tj = jc / kTile, qj = jc % kTile;
    const double al = in_tile[tj].alpha;
    const float aj = in_A[jc];
    double na = 0.0, ab = 0.0, gb = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double ad = (double)P[d] - (double)in_tile[tj].ctr[d];
      const double bd = (double)in_off[((size_t)tj * D + d) * kTile + qj];
      na += ad * ad;
      ab += ad * bd;
      gb += (double)in_tile[tj].gam[d] * bd;
    }
    if (j >= 0 && j < count_in && al > -INFINITY && aj > -INFINITY) {
      M = al + (double)aj + gb + kap2d * (2.0 * ab - na);
      J = j;
    }
  }
  // the records' reference: the warm start's exponent (the same in every
  // split), 0 without one; split 0 stores it for the merge
  const double Rref = M > -INFINITY ? M : 0.0;
  if (!BARY && split == 0) part_ref[p] = Rref;
  float S = 0.0f, N = 0.0f;
  float V[D];
  // writes this split's record: the shift relative to the reference in
  // float32, the sums rescaled by that rounding so that the record is exact
  auto write_rec = [&]() {
    float dM = -INFINITY, fix = 1.0f;
    if (M > -INFINITY) {
      const double dd = M - Rref;
      dM = (float)dd;
      fix = fast_exp2((float)(dd - (double)dM));
    }
    if (CERT) {
      reinterpret_cast<PartialCert*>(part)[(size_t)split * np_out + p] = PartialCert{dM, S * fix, N * fix, J};
    } else {
      reinterpret_cast<PartialRec*>(part)[(size_t)split * np_out + p] = PartialRec{dM, S * fix, J};
    }
  };
#pragma unroll
  for (int d = 0; d < D; ++d) V[d] = 0.0f;
  int evaluated = 0;  // input tiles this wavefront evaluated (the same on every lane)
  if (nt == 0) {
    if (tile_count && (threadIdx.x & (kTile - 1)) == 0) tile_count[slot] = 0;
    if (BARY) {
      PartialBary* pb = reinterpret_cast<PartialBary*>(part) + (size_t)split * np_out + p;
      pb->M = M;
      pb->S = S;
      for (int d = 0; d < 3; ++d) pb->V[d] = 0.0f;
    } else {
      write_rec();
    }
    return;
  }

  const double tskip = skip_threshold(count_in);
  double Mth = M + kThresh;                     // the exact-max gate, updated with M
  double Mlo = M - tskip;                       // the skip gate, updated with M
  // The weights are read with broadcast vector loads (a lane-dependent zero in
  // the address), which leaves the scalar path to the offsets and the
  // candidates' tile records: moving either kind the other way measured slower.
  Group<D> grp;
  for (int c0 = 0; c0 < nt; c0 += kTile) {
    const int c1 = min(c0 + kTile, nt);
    if (c0 != 0) cub = coarse(c0, c1);
    const double mlo_min = -wave_max(-Mlo);
    unsigned long long cand = __ballot(c0 + lane < c1 && !(cub < mlo_min));
    if (cand) {
      const int tf = split + (c0 + __builtin_ctzll(cand)) * nsplit;
      grp = load_group<D>(in_off + (size_t)tf * D * kTile, in_A + (size_t)tf * kTile + lane0, 0);
    }
    while (cand) {
      const int t = split + (c0 + __builtin_ctzll(cand)) * nsplit;
      cand &= cand - 1;
      const TileVals<D> cur = load_tile<D>(in_tile + t);
      const int tn = cand ? split + (c0 + __builtin_ctzll(cand)) * nsplit : t;  // next candidate (the last re-reads itself)
      // tile addresses computed before any lane-dependent branch
      gfloat* __restrict__ offs_t = in_off + (size_t)t * D * kTile;
      gfloat* __restrict__ a_t = in_A + (size_t)t * kTile + lane0;
      gfloat* __restrict__ offs_n = in_off + (size_t)tn * D * kTile;
      gfloat* __restrict__ a_n = in_A + (size_t)tn * kTile + lane0;
      float a[D];
#pragma unroll
      for (int d = 0; d < D; ++d) a[d] = P[d] - cur.ctr[d];
      // upper bound of the exponents w2_q - kappa2 |a - b_q|^2 of this tile:
      // w2_q <= alpha + gamma . b_q + rho, and the concave quadratic
      // gamma . b - kappa2 |a - b|^2 is maximised over the tile's box per axis
      float ubf = cur.rho;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const float g = cur.gam[d], rad = cur.rad[d];
        const float bs = __builtin_amdgcn_fmed3f(fmaf(g, inv2kap, a[d]), -rad, rad);  // clamp to the box
        const float df = a[d] - bs;
        ubf = fmaf(g, bs, ubf);
        ubf = fmaf(-kap2f, df * df, ubf);
      }
      const double ub = cur.alpha + (double)ubf;
      // every term of this tile lies below 2^-T of the running maximum on every
      // lane: the tile cannot change any sum in float32, so it is skipped.  A
      // tile without mass (alpha = -inf) is skipped here once M is finite, and
      // by its maximum below; testing the maximum first would make every tile
      // wait for two scalar round trips (the maximum, then the bound's fields)
      if (__all(ub < Mlo) ||
          __double_as_longlong(cur.amax) == (long long)0xFFF0000000000000ULL) {  // -inf: no mass
        grp = load_group<D>(offs_n, a_n, 0);
        continue;
      }
      ++evaluated;
      float B[D], na = 0.0f;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        na = fmaf(a[d], a[d], na);
        B[d] = (float)fma(kap2x2d, (double)a[d], (double)cur.gam[d]);  // gamma + 2 kappa2 a, rounded once
      }
      const double base = cur.alpha - kap2d * (double)na;  // alpha_t - kappa2 |a|^2

      if (ub > Mth) {
        // exact maximum of this tile for the lanes whose bound exceeds the window
        gfloat* __restrict__ offs = offs_t;
        gfloat* __restrict__ Aq = a_t;
        float tm = -INFINITY;
        int qi = 0;
#pragma unroll 8
        for (int q = 0; q < kTile; ++q) {
          float z = Aq[q];
#pragma unroll
          for (int d = 0; d < D; ++d) z = fmaf(B[d], offs[d * kTile + q], z);
          if (z > tm) {
            tm = z;
            qi = q;
          }
        }
        const double tmd = base + (double)tm;
        if (tmd > M) {
          const float sc = fast_exp2((float)(M - tmd));
          S *= sc;
          if (CERT) N *= sc;
          if (BARY) {
#pragma unroll
            for (int d = 0; d < D; ++d) V[d] *= sc;
          }
          M = tmd;
          Mth = M + kThresh;
          Mlo = M - tskip;
          J = t * kTile + qi;
        }
      }
      const float cm = (float)(base - M);
      float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
      float n0 = 0.f, n1 = 0.f;
      float vt[D];
#pragma unroll
      for (int d = 0; d < D; ++d) vt[d] = 0.0f;
#pragma unroll
      for (int g = 0; g < kTile / kGroup; ++g) {
        // request the next group (the first group of the next tile after the last)
        const Group<D> nx = (g + 1 < kTile / kGroup) ? load_group<D>(offs_t, a_t, g + 1)
                                                    : load_group<D>(offs_n, a_n, 0);
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
          float z = cm;
#pragma unroll
          for (int d = 0; d < D; ++d) z = fmaf(B[d], grp.b[d][u], z);
          z += grp.a[u];
          const float e = fast_exp2(z);
          if (g == 0 && u < 4) {
            (u == 0 ? s0 : u == 1 ? s1 : u == 2 ? s2 : s3) = e;
          } else {
            (u % 4 == 0 ? s0 : u % 4 == 1 ? s1 : u % 4 == 2 ? s2 : s3) += e;
          }
          if (CERT) {
            float c2 = 0.0f;
#pragma unroll
            for (int d = 0; d < D; ++d) {
              const float df = a[d] - grp.b[d][u];
              c2 = fmaf(df, df, c2);
            }
            if (u & 1) n1 = fmaf(c2, e, n1); else n0 = fmaf(c2, e, n0);
          }
          if (BARY) {
#pragma unroll
            for (int d = 0; d < D; ++d) vt[d] = fmaf(e, grp.b[d][u], vt[d]);
          }
        }
        grp = nx;
      }
      const float st = (s0 + s1) + (s2 + s3);
      S += st;
      if (CERT) N += n0 + n1;
      if (BARY) {
        // sum_q e_q y_q = c_t sum_q e_q + sum_q e_q b_q (points = tile centre + offset)
#pragma unroll
        for (int d = 0; d < D; ++d) V[d] += fmaf(cur.ctr[d], st, vt[d]);
      }
    }
  }
  if (tile_count && (threadIdx.x & (kTile - 1)) == 0) tile_count[slot] = (unsigned)evaluated;
  if (BARY) {
    PartialBary* pb = reinterpret_cast<PartialBary*>(part) + (size_t)split * np_out + p;
    pb->M = M;
    pb->S = S;
    for (int d = 0; d < 3; ++d) pb->V[d] = d < D ? V[d] : 0.0f;
    return;
  }
  write_rec();
}

template <int D, int MODE>
__global__ __launch_bounds__(kSweepBlock) void k_sweep(
    const float* __restrict__ out_abs, int np_out,
    const float* __restrict__ in_off, const float* __restrict__ in_A, const TileRec* __restrict__ in_tile,
    int ntiles_in, int count_in, int nsplit, const int* __restrict__ hint,
    void* __restrict__ part, double* __restrict__ part_ref, const Ctrl* __restrict__ ctrl, double eps_arg, int kofs,
    int row_sweep, unsigned* __restrict__ tile_count) {
  // blockIdx.x is the split and blockIdx.y the output block: consecutive
  // workgroups go to consecutive XCDs, so the splits of one output block
  // spread over all XCDs (a heavy output region does not load one XCD) and
  // each XCD reads the input tiles of only splits / 8 splits (its L2 holds
  // just those)
  const int slot = (blockIdx.y * gridDim.x + blockIdx.x) * (kSweepBlock / kTile) + threadIdx.x / kTile;
  sweep_block<D, MODE>((gfloat*)out_abs, np_out, (gfloat*)in_off, (gfloat*)in_A, (gtile*)in_tile, ntiles_in,
                       count_in, nsplit, hint, part, part_ref, (gctrl*)ctrl, eps_arg, kofs, blockIdx.y, blockIdx.x,
                       row_sweep != 0, tile_count, slot);
}

// Batched sweep: block i runs work item i = (problem, block of outputs, split)
// of a list over several problems; the arithmetic per item is the same as in
// the single-problem launch.
template <int D, int MODE>
__global__ __launch_bounds__(kSweepBlock) void k_sweep_batch(const BatchItem* __restrict__ items,
                                                        const LaunchCtx* __restrict__ descs, int transpose,
                                                        int kofs) {
  const BatchItem it = items[blockIdx.x];
  const LaunchCtx& c = descs[it.prob];
  const SideDev& out = transpose ? c.cols : c.rows;
  const SideDev& in = transpose ? c.rows : c.cols;
  const int splits = transpose ? c.splits_col : c.splits_row;
  sweep_block<D, MODE>((gfloat*)out.abs, out.np, (gfloat*)in.off, (gfloat*)in.A, (gtile*)in.tile, in.ntiles,
                       in.count, splits, out.hint, c.part.rec, c.part.ref, (gctrl*)c.ctrl, -1.0, kofs, it.blk, it.split,
                       transpose == 0, nullptr, 0);
}

// ---------------------------------------------------------------------------
// Finish: merge the split partials (float64) and run the epilogue.
// ---------------------------------------------------------------------------
struct Merged {
  double lse;   // natural-log LSE
  double S;     // merged shifted sum (relative to Mx)
  double N;     // merged shifted cost sum
  int J;        // input slot of the exact maximum of the winning split, or -1
};

template <typename Rec>
__device__ __forceinline__ float rec_N(const Rec& q) { return 0.0f; }
template <>
__device__ __forceinline__ float rec_N<PartialCert>(const PartialCert& q) { return q.N; }

template <typename Rec>
__device__ __forceinline__ Merged merge_splits_t(const Rec* __restrict__ part, const double* __restrict__ ref,
                                                 int splits, int np, int p) {
  // The epilogue runs few waves, so its time is the number of memory round
  // trips: one pass over the split records, G of them requested together.
  // Past the last split the index is clamped to a valid record and its shift
  // gets -inf added (so its weight is 0): every loaded value is used
  // unconditionally, which keeps the loads together (a load the compiler may
  // sink under a branch waits for its data before the next one is issued).
  // Each batch is merged against the running maximum, which is raised first
  // if the batch holds a larger one (the running sums are rescaled).  Shifts
  // are relative to the output's reference R.
  constexpr int G = 16;
  const double R = ref[p];
  float mx = -INFINITY;
  double S = 0.0, N = 0.0;
  int J = -1;
  auto batch = [&](int s0) {
    Rec q[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      q[g] = part[(size_t)min(s0 + g, splits - 1) * np + p];
      q[g].dM += (s0 + g < splits) ? 0.0f : -INFINITY;
    }
    float bm = -INFINITY;
    int bj = -1;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const bool up = q[g].dM > bm;  // the first split holding the batch maximum
      bj = up ? q[g].J : bj;
      bm = up ? q[g].dM : bm;
    }
    if (bm > mx) {  // strictly: J stays with the first split holding the maximum
      // shifts of one output differ by little: the weight is a hardware float32 exp2
      const double sc = mx == -INFINITY ? 0.0 : (double)fast_exp2(mx - bm);
      S *= sc;
      N *= sc;
      mx = bm;
      J = bj;
    }
    if (mx == -INFINITY) return;  // nothing so far
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const double w = (double)fast_exp2(q[g].dM - mx);  // 0 for an empty or masked split
      S += w * (double)q[g].S;
      N += w * (double)rec_N(q[g]);
    }
  };
  // the first batch outside the loop: at a loop header the wait counts are
  // merged conservatively, which would wait for the loads issued before it
  batch(0);
  for (int s0 = G; s0 < splits; s0 += G) batch(s0);
  Merged r{-INFINITY, 0.0, 0.0, -1};
  if (mx == -INFINITY) return r;  // empty sum
  r.S = S;
  r.N = N;
  r.J = J;
  r.lse = kLn2D * ((R + (double)mx) + log2(S));
  return r;
}

__device__ __forceinline__ Merged merge_splits(const Partials& pt, bool cert, int splits, int np, int p) {
  if (cert) return merge_splits_t(reinterpret_cast<const PartialCert*>(pt.rec), pt.ref, splits, np, p);
  return merge_splits_t(reinterpret_cast<const PartialRec*>(pt.rec), pt.ref, splits, np, p);
}

// Packs the weights w of one tile for the sweeps: a least-squares plane
// w2 ~ alpha + gamma . b of the tile's log2 weights w2 = log2(e) w over the
// offsets b, with its largest residual rho (so w2 <= alpha + gamma . b + rho
// holds for every point of the tile, whatever the fit: the sweep turns it
// into an upper bound of its exponents), and per point
// A_p = w2_p - alpha - gamma . b_p - kappa2 |b_p|^2 in float32 (-inf on padding
// or for w = -inf), the part of the exponent that does not depend on the
// output.  The record also holds the tile maximum of w2 - kappa2 |b|^2
// (float64; -inf when the tile has no mass).  Called by whole wavefronts (one
// tile each).
// Offsets of point p from its tile centre (0 past the real points); the
// epilogues request them before they wait for the split records.
// Three loads at clamped (valid) addresses whatever dim and p are, zeroed by a
// multiplication (offsets are finite) rather than a select, so that every
// loaded value is used and the loads issue together.
__device__ __forceinline__ void load_offsets(const SideDev& sd, int dim, int p, float bo[3]) {
  const int t = min(p, sd.count - 1) / kTile, q = p % kTile;
  const float* base = sd.off + (size_t)t * dim * kTile + q;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float v = base[(size_t)min(d, dim - 1) * kTile];
    bo[d] = v * ((p < sd.count && d < dim) ? 1.0f : 0.0f);
  }
}

template <int D>
__device__ __forceinline__ void pack_weight_d(const SideDev& sd, int p, double w, double kap2, const float bo[3]) {
  constexpr int dim = D;
  const bool live = p < sd.count && w > -INFINITY;
  const int t = p / kTile;
  double A = -INFINITY, w2 = 0.0;
  double b[D];
  float n2 = 0.0f;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    b[d] = (double)bo[d];
    n2 = fmaf(bo[d], bo[d], n2);
  }
  if (live) {
    w2 = kLog2eD * w;
    A = w2 - kap2 * (double)n2;
  }
  if (p >= sd.ntiles * kTile) return;
  const double m = wave_max(A);
  double gam[3] = {0.0, 0.0, 0.0}, alpha = -INFINITY;
  // least-squares plane through the live points of the tile (centred sums).
  // When the live points are the tile's real points (every weight finite, as
  // in the iterations: the marginals are positive), their geometry is the
  // tile's precomputed one and the fit needs only the sums of w2 and of the
  // centred offsets times w2 (the centred offsets sum to zero, so the latter
  // is the centred cross sum), all taken at once.
  const int nreal = min(kTile, sd.count - t * kTile);
  const unsigned long long real_mask = nreal >= kTile ? ~0ull : ((1ull << nreal) - 1ull);
  if (__ballot(live) == real_mask) {
    const TileGeom* g = sd.geom + t;
    const double wl = live ? w2 : 0.0;
    double v[D + 1];
    v[0] = wl;
#pragma unroll
    for (int d = 0; d < D; ++d) v[d + 1] = live ? (b[d] - g->mb[d]) * wl : 0.0;
    wave_sum_n<D + 1>(v);
    const double mw = v[0] / g->cnt;
    // symmetric inverse stored as xx, xy, xz, yy, yz, zz
    constexpr int kSym[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    alpha = mw;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      double s = 0.0;
#pragma unroll
      for (int e = 0; e < D; ++e) s = fma(g->cinv[kSym[d][e]], v[e + 1], s);
      gam[d] = (double)(float)s;  // the sweep reads gamma as float32
      alpha -= gam[d] * g->mb[d];
    }
  } else {
    const double one = live ? 1.0 : 0.0;
    const double cnt = wave_sum(one);
    double mb[D], mw = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) mb[d] = 0.0;
    if (cnt > 0.0) {
      for (int d = 0; d < dim; ++d) mb[d] = wave_sum(one * b[d]) / cnt;
      mw = wave_sum(live ? w2 : 0.0) / cnt;
      double cbb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, cbw[3] = {0, 0, 0};
      for (int d = 0; d < dim; ++d) {
        const double bd = live ? b[d] - mb[d] : 0.0;
        cbw[d] = wave_sum(bd * (live ? w2 - mw : 0.0));
        for (int e = 0; e <= d; ++e) {
          cbb[d][e] = wave_sum(bd * (live ? b[e] - mb[e] : 0.0));
          cbb[e][d] = cbb[d][e];
        }
      }
      // solve cbb gamma = cbw by Cramer's rule; a (near-)singular system keeps gamma = 0
      if constexpr (D == 1) {
        if (cbb[0][0] > 1e-12) gam[0] = cbw[0] / cbb[0][0];
      } else if constexpr (D == 2) {
        const double det = cbb[0][0] * cbb[1][1] - cbb[0][1] * cbb[1][0];
        if (fabs(det) > 1e-12 * (cbb[0][0] * cbb[1][1] + 1e-300)) {
          gam[0] = (cbw[0] * cbb[1][1] - cbb[0][1] * cbw[1]) / det;
          gam[1] = (cbb[0][0] * cbw[1] - cbw[0] * cbb[1][0]) / det;
        }
      } else {
        const double a00 = cbb[1][1] * cbb[2][2] - cbb[1][2] * cbb[2][1];
        const double a01 = cbb[0][2] * cbb[2][1] - cbb[0][1] * cbb[2][2];
        const double a02 = cbb[0][1] * cbb[1][2] - cbb[0][2] * cbb[1][1];
        const double det = cbb[0][0] * a00 + cbb[1][0] * a01 + cbb[2][0] * a02;
        if (fabs(det) > 1e-12 * (cbb[0][0] * cbb[1][1] * cbb[2][2] + 1e-300)) {
          const double a10 = cbb[1][2] * cbb[2][0] - cbb[1][0] * cbb[2][2];
          const double a11 = cbb[0][0] * cbb[2][2] - cbb[0][2] * cbb[2][0];
          const double a12 = cbb[0][2] * cbb[1][0] - cbb[0][0] * cbb[1][2];
          const double a20 = cbb[1][0] * cbb[2][1] - cbb[1][1] * cbb[2][0];
          const double a21 = cbb[0][1] * cbb[2][0] - cbb[0][0] * cbb[2][1];
          const double a22 = cbb[0][0] * cbb[1][1] - cbb[0][1] * cbb[1][0];
          gam[0] = (a00 * cbw[0] + a01 * cbw[1] + a02 * cbw[2]) / det;
          gam[1] = (a10 * cbw[0] + a11 * cbw[1] + a12 * cbw[2]) / det;
          gam[2] = (a20 * cbw[0] + a21 * cbw[1] + a22 * cbw[2]) / det;
        }
      }
      for (int d = 0; d < dim; ++d) gam[d] = (double)(float)gam[d];  // the sweep reads gamma as float32
      alpha = mw;
      for (int d = 0; d < dim; ++d) alpha -= gam[d] * mb[d];
    }
  }
  double res = 0.0;
  if (live) {
    res = w2 - alpha;
    for (int d = 0; d < dim; ++d) res -= gam[d] * b[d];
  }
  // the weight's residual from the plane minus the tile-local quadratic
  sd.A[p] = live ? (float)(res - kap2 * (double)n2) : -INFINITY;
  const double rho = wave_max(fabs(res));
  if ((threadIdx.x & (kTile - 1)) == 0) {
    TileRec& tr = sd.tile[t];
    tr.amax = m;
    tr.alpha = alpha;
    for (int d = 0; d < 3; ++d) tr.gam[d] = (float)gam[d];
    tr.rho = (float)(rho * (1.0 + 1e-6)) + 1e-3f;  // rounded up: the bound must hold
  }
}

__device__ __forceinline__ void pack_weight(const SideDev& sd, int dim, int p, double w, double kap2,
                                            const float bo[3]) {
  if (dim == 1) pack_weight_d<1>(sd, p, w, kap2, bo);
  else if (dim == 2) pack_weight_d<2>(sd, p, w, kap2, bo);
  else pack_weight_d<3>(sd, p, w, kap2, bo);
}

__device__ __forceinline__ void pack_weight(const SideDev& sd, int dim, int p, double w, double kap2) {
  float bo[3];
  load_offsets(sd, dim, p, bo);
  pack_weight(sd, dim, p, w, kap2, bo);
}

// Merge of the barycentric partials of output p: shift, shifted sum and the
// shifted coordinate sums, in float64.
struct MergedBary {
  double lse;   // natural-log LSE
  double V[3];  // coordinate sums relative to the merged sum
};

__device__ __forceinline__ MergedBary merge_bary(const void* __restrict__ part, int splits, int np, int p) {
  const PartialBary* pb = reinterpret_cast<const PartialBary*>(part);
  double mx = -INFINITY;
  for (int s = 0; s < splits; ++s) mx = fmax(mx, pb[(size_t)s * np + p].M);
  MergedBary r;
  double S = 0.0, V[3] = {0.0, 0.0, 0.0};
  if (mx > -INFINITY) {
    for (int s = 0; s < splits; ++s) {
      const PartialBary q = pb[(size_t)s * np + p];
      const double w = exp2(q.M - mx);
      S += w * (double)q.S;
      for (int d = 0; d < 3; ++d) V[d] += w * (double)q.V[d];
    }
  }
  r.lse = kLn2D * (mx + log2(S));
  for (int d = 0; d < 3; ++d) r.V[d] = S > 0.0 ? V[d] / S : 0.0;
  return r;
}

// Merge + epilogue of one tile (bx) of 64 outputs; nblocks = tiles of the
// output side (the column epilogue's last block advances k).
__device__ __forceinline__ void finish_block(const LaunchCtx& c, int transpose, int kind, int splits,
                                             double eps_arg, double* __restrict__ lse_out, int bx, int kofs) {
  const SideDev& out = transpose ? c.cols : c.rows;
  const int p = bx * kTile + threadIdx.x;
  const int np = out.np;
  if (p >= np) return;
  const bool real = p < out.count;
  if (kind == kFinishPlanRow) {
    // state plan: (X 1)_i = alpha_i sum_j K_ij beta_j, barycentre sum_j X_ij y_j / (X 1)_i
    const MergedBary mb = merge_bary(c.part.rec, splits, np, p);
    if (real) {
      c.plan_row[p] = exp(c.st.la[p] + mb.lse);
      if (lse_out) {
        const int i = out.perm[p];
        for (int d = 0; d < c.dim; ++d) lse_out[(size_t)i * c.dim + d] = c.origin[d] + mb.V[d];
      }
    }
    return;
  }
  const bool cert = (kind == kFinishColCert || kind == kFinishCertOnly);
  const bool iter_kind = kind == kFinishRow || kind == kFinishCol || kind == kFinishColCert;
  // An epilogue runs one wavefront per output tile, so its time is the number
  // of memory round trips: what the iteration's epilogues read that does not
  // depend on the merge (control block, marginal, dual state, the offsets the
  // packing needs) is requested before the split records are waited for.
  // Unconditional loads (p < np, and every array read here holds np entries
  // of the output side): a load under a branch is waited for there.
  const Ctrl cv = *c.ctrl;
  float bo[3];
  load_offsets(out, c.dim, p, bo);
  const double* s_arr = transpose ? c.st.lb1 : c.st.la;
  const double* t0_arr = transpose ? c.st.lt[0] : c.st.la;
  const double* t1_arr = transpose ? c.st.lt[1] : c.st.la;
  const double pre_lm = out.logmarg[p], pre_s = s_arr[p], pre_t0 = t0_arr[p], pre_t1 = t1_arr[p];
  // the sweeps that gathered cost-weighted sums wrote certificate records
  const bool cert_rec = kind == kFinishColCert || kind == kFinishCertOnly || kind == kFinishRound3;
  const Merged mg = merge_splits(c.part, cert_rec, splits, np, p);
  // the warm start of the next sweep of this side: only the iteration's own sweeps set it
  if (real && iter_kind && mg.J >= 0) out.hint[p] = mg.J;
  const Ctrl* ctrl = &cv;
  const long long k = ctrl->k + kofs;  // this iteration: the block's first plus the offset
  const double lam = ctrl->lam;

  if (kind == kFinishLse) {
    if (real) lse_out[out.perm[p]] = mg.lse;
    return;
  }
  if (kind == kFinishPlanCol) {
    // (X^T 1)_j = beta_j sum_i K_ij alpha_i
    if (real) c.plan_col[p] = exp(c.st.lb1[p] + mg.lse);
    return;
  }
  // two-sided rounding of the state plan (Altschuler, Weed and Rigollet 2017, Algorithm 2)
  if (kind == kFinishRound1) {
    // log x_i = min(0, log r_i - log (X 1)_i)
    if (real) c.plan_row[p] = fmin(0.0, out.logmarg[p] - (c.st.la[p] + mg.lse));
    return;
  }
  if (kind == kFinishRound2) {
    // X' = diag(x) X: log y_j = min(0, log c_j - log (X'^T 1)_j); deficit c_j - y_j (X'^T 1)_j
    if (real) {
      const double lcol = c.st.lb1[p] + mg.lse;
      const double ly = fmin(0.0, out.logmarg[p] - lcol);
      c.plan_col[p] = ly;
      // nonnegative by construction; the clamp removes an ulp of rounding
      // where y_j = c_j / (X'^T 1)_j, so that every entry of G is >= 0
      c.st.mu[p] = fmax(0.0, out.marg[p] - exp(lcol + ly));
    }
    return;
  }
  if (kind == kFinishRound3) {
    // X'' = diag(x) X diag(y): row deficit r_i - (X'' 1)_i and sum_j X''_ij C_ij
    if (real) {
      const double row2 = exp(c.st.la[p] + c.plan_row[p] + mg.lse);
      c.plan_aux[p] = fmax(0.0, out.marg[p] - row2);
      c.st.pvec[p] = row2 * ctrl->scale * mg.N / mg.S;
    }
    return;
  }
  if (kind == kFinishCertOnly) {
    // Algorithm 2 for the last finished iteration k-1 (k has been advanced)
    if (real) {
      c.st.mu[p] = ctrl->scale * mg.N / mg.S;
      c.st.logs[p] = c.st.lt[(k - 1) & 1][p] + mg.lse;
    }
    return;
  }
  if (kind == kFinishRepair) {
    // p_i = A_i sum_j K_ij t_j (1 - e_j) = exp(log alpha-hat_i + LSE_i)
    c.st.pvec[p] = real ? exp(c.st.lah[p] + mg.lse) : 0.0;
    return;
  }
  if (kind == kFinishRow) {
    // row update of Algorithm 1: the unrelaxed row scaling normalises the rows to r; the
    // relaxed one mixes it with the previous relaxed scaling, weight lambda on the new one
    const double eps = eps_of(ctrl, eps_arg, kofs);
    const double kap2 = kLog2eD * ctrl->scale / eps;
    double colw = 0.0;
    if (real) {
      const double lah = pre_lm - mg.lse;
      c.st.lah[p] = lah;
      if (ctrl->variant & kVarDebiased) {
        // debiased row update: log a^k = theta_k log a^{k-1} + log r - LSE, theta_k = 0 (k <= 1), 1/k
        const double theta = k <= 1 ? 0.0 : 1.0 / (double)k;
        colw = theta * pre_s + lah;
        c.st.la[p] = colw;
      } else {
        // one rounded product fused into the other: fixed whatever the
        // compiler's contraction (the result is exact for lambda = 1)
        c.st.la[p] = fma(lam, lah, (1.0 - lam) * pre_s);
        colw = lah;
      }
    }
    // weights of the column sweep of the same iteration: log alpha-hat (the
    // debiased variant: its row scaling a^k)
    pack_weight(c.rows, c.dim, p, colw, kap2, bo);
    return;
  }
  // column epilogue (plain or certificate)
  const int cur = (int)(k & 1), nxt = (int)((k + 1) & 1);
  double lt_next = 0.0;
  if (real) {
    const double lbh = pre_lm - mg.lse;                 // log beta-hat^k = log c - LSE
    const double lb1 = pre_s;
    const double lb = fma(lam, lbh, (1.0 - lam) * lb1);  // log beta^k (rounding as for alpha)
    if (cert) {
      // certificate statistics of the intermediate plan's column (Prop. 3, Algorithm 2):
      // its mean cost (cost-weighted over plain merged sums) and the log of its mass
      c.st.mu[p] = ctrl->scale * mg.N / mg.S;
      c.st.logs[p] = (cur ? pre_t1 : pre_t0) + mg.lse;
    }
    c.st.lbh[p] = lbh;
    c.st.lb2[p] = lb1;
    c.st.lb1[p] = lb;
    // momentum for iteration k+1: log beta-tilde^k = log beta^k + (log beta^k - log beta^{k-1}) / lambda
    lt_next = (ctrl->variant & kVarNoMomentum) ? lb : lb + (lb - lb1) / lam;
    c.st.lt[nxt][p] = lt_next;
  }
  const double eps1 = eps_row_of(ctrl, -1.0, kofs + 1);
  const double kap2n = kLog2eD * ctrl->scale / eps1;
  pack_weight(c.cols, c.dim, p, lt_next, kap2n, bo);

}

__global__ __launch_bounds__(kTile) void k_finish(LaunchCtx c, int transpose, int kind, int splits,
                                                  double eps_arg, double* __restrict__ lse_out, int kofs) {
  finish_block(c, transpose, kind, splits, eps_arg, lse_out, blockIdx.x, kofs);
}

// Advances the iteration counter by n after a block of n iterations (kernels of
// the block read the block's first iteration and take their offset as an
// argument, so a captured block replays at any k).
__global__ void k_advance(Ctrl* ctrl, int n) {
  if (threadIdx.x == 0) ctrl->k += n;
}

__global__ void k_advance_batch(const LaunchCtx* __restrict__ descs, int count, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) descs[i].ctrl->k += n;
}

// Batched merge + epilogue: block i runs item i = (problem, output tile).
__global__ __launch_bounds__(kTile) void k_finish_batch(const BatchItem* __restrict__ items,
                                                        const LaunchCtx* __restrict__ descs, int transpose,
                                                        int kind, int kofs) {
  const BatchItem it = items[blockIdx.x];
  const LaunchCtx& c = descs[it.prob];
  finish_block(c, transpose, kind, transpose ? c.splits_col : c.splits_row, -1.0, nullptr, it.blk, kofs);
}

// lt and A_C of iteration k from the stored log beta^{k-1}, log beta^{k-2}.
__global__ __launch_bounds__(kBlock) void k_prologue(LaunchCtx c) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= c.cols.np) return;
  const long long k = c.ctrl->k;
  const double lam = c.ctrl->lam;
  const bool real = p < c.cols.count;
  double lt = 0.0;
  if (real) {
    const double lb1 = c.st.lb1[p], lb2 = c.st.lb2[p];
    lt = (c.ctrl->variant & kVarNoMomentum) ? lb1 : lb1 + (lb1 - lb2) / lam;
    c.st.lt[k & 1][p] = lt;
  }
  const double kap2 = kLog2eD * c.ctrl->scale / eps_row_of(c.ctrl, -1.0, 0);
  pack_weight(c.cols, c.dim, p, lt, kap2);
}

// A of the input side from caller weights w (original order), for bdrs_lse.
__global__ __launch_bounds__(kBlock) void k_pack(LaunchCtx c, int transpose, const double* __restrict__ w,
                                                 double eps) {
  const SideDev& in = transpose ? c.rows : c.cols;
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= in.np) return;
  const double kap2 = kLog2eD * c.ctrl->scale / eps;
  const double wv = p < in.count ? w[in.perm[p]] : 0.0;
  pack_weight(in, c.dim, p, wv, kap2);
}

// rows.A from the stored log alpha-hat (re-pack after the sweep buffers were reused).
__global__ __launch_bounds__(kBlock) void k_pack_rows(LaunchCtx c, double eps) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= c.rows.np) return;
  const double kap2 = kLog2eD * c.ctrl->scale / eps;
  pack_weight(c.rows, c.dim, p, p < c.rows.count ? c.st.lah[p] : 0.0, kap2);
}

// State-plan weights of the input side: log beta^{k-1} on the columns (row sums
// and barycentres), log alpha^{k-1} on the rows (column sums), at temperature eps.
__global__ __launch_bounds__(kBlock) void k_pack_state(LaunchCtx c, int transpose, double eps, int with_factors) {
  const SideDev& in = transpose ? c.rows : c.cols;
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= in.np) return;
  const double kap2 = kLog2eD * c.ctrl->scale / eps;
  const double* w = transpose ? c.st.la : c.st.lb1;
  const double* f = transpose ? c.plan_row : c.plan_col;
  double v = 0.0;
  if (p < in.count) v = with_factors ? w[p] + f[p] : w[p];
  pack_weight(in, c.dim, p, v, kap2);
}

// Marginal-error statistics of the state plan (float64): per block partial
// sums / maxima over both sides, then one block combines them in order.
// Partial layout per block: row l1, row max abs, row max rel, col l1, col max
// abs, col max rel, total mass, pad.
__global__ __launch_bounds__(kBlock) void k_plan_partial(LaunchCtx c) {
  __shared__ double sh[kBlock / kTile][8];
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int stride = gridDim.x * kBlock;
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < c.rows.count; p += stride) {
    const double r = c.rows.marg[p], x = c.plan_row[p];
    const double e = fabs(x - r);
    v[0] += e;
    v[1] = fmax(v[1], e);
    v[2] = fmax(v[2], e / r);
    v[6] += x;
  }
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < c.cols.count; p += stride) {
    const double cj = c.cols.marg[p];
    const double e = fabs(c.plan_col[p] - cj);
    v[3] += e;
    v[4] = fmax(v[4], e);
    v[5] = fmax(v[5], e / cj);
  }
  v[0] = wave_sum(v[0]);
  v[3] = wave_sum(v[3]);
  v[6] = wave_sum(v[6]);
  v[1] = wave_max(v[1]);
  v[2] = wave_max(v[2]);
  v[4] = wave_max(v[4]);
  v[5] = wave_max(v[5]);
  const int wv = threadIdx.x / kTile;
  if ((threadIdx.x & (kTile - 1)) == 0)
    for (int i = 0; i < 8; ++i) sh[wv][i] = v[i];
  __syncthreads();
  if (threadIdx.x < 8) {
    const int i = threadIdx.x;
    double a = sh[0][i];
    for (int w = 1; w < kBlock / kTile; ++w) a = (i == 0 || i == 3 || i == 6) ? a + sh[w][i] : fmax(a, sh[w][i]);
    c.cert_part[(size_t)blockIdx.x * 8 + i] = a;
  }
}

__global__ __launch_bounds__(kBlock) void k_plan_final(LaunchCtx c, int nblocks) {
  if (threadIdx.x < 8) {
    const int i = threadIdx.x;
    double a = c.cert_part[i];
    for (int b = 1; b < nblocks; ++b) {
      const double x = c.cert_part[(size_t)b * 8 + i];
      a = (i == 0 || i == 3 || i == 6) ? a + x : fmax(a, x);
    }
    c.plan_stats[i] = a;
  }
}

// Repair weights: log t_j + log(1 - e_j), e_j = min(1, c_j / s_j) (-inf where e_j = 1).
__global__ __launch_bounds__(kBlock) void k_repair_pack(LaunchCtx c) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= c.cols.np) return;
  const long long k = c.ctrl->k - 1;  // the certified iteration
  double w = -INFINITY;
  if (p < c.cols.count) {
    const double s = exp(c.st.logs[p]);
    const double cj = c.cols.marg[p];
    if (s > cj) w = c.st.lt[k & 1][p] + log1p(-cj / s);
  }
  const double kap2 = kLog2eD * c.ctrl->scale / eps_row_of(c.ctrl, -1.0, -1);
  pack_weight(c.cols, c.dim, p, w, kap2);
}

// ---------------------------------------------------------------------------
// Certificate reductions (float64).  Partial sums per block, then one block
// adds the partials in a fixed order (deterministic).
// slots: 0 sum r log A, 1 sum c (log B - log c), 2 sum |s - c|, 3 sum s mu,
//        4 sum s, 5 non-finite count
// ---------------------------------------------------------------------------
__device__ void block_reduce_store(double* vals, int nv, double* dst) {
  __shared__ double red[kBlock / kTile][8];
  const int lane = threadIdx.x & (kTile - 1), wid = threadIdx.x / kTile;
  for (int i = 0; i < nv; ++i) {
    const double v = wave_sum(vals[i]);
    if (lane == 0) red[wid][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    double s = 0.0;
    for (int w = 0; w < kBlock / kTile; ++w) s += red[w][threadIdx.x];
    dst[threadIdx.x] = s;
  }
}

__device__ __forceinline__ void cert_partial_block(const LaunchCtx& c, int bx, int nb) {
  double v[6] = {0, 0, 0, 0, 0, 0};
  const int stride = nb * kBlock;
  const bool debiased = (c.ctrl->variant & kVarDebiased) != 0;
  for (int p = bx * kBlock + threadIdx.x; p < c.rows.count; p += stride) {
    // f = eps log A with A the row scaling the column update read (Prop. 3)
    const double lah = debiased ? c.st.la[p] : c.st.lah[p];
    if (!isfinite(lah)) v[5] += 1.0;
    v[0] += c.rows.marg[p] * lah;
  }
  for (int p = bx * kBlock + threadIdx.x; p < c.cols.count; p += stride) {
    const double lbh = c.st.lbh[p];
    const double cj = c.cols.marg[p];
    const double s = exp(c.st.logs[p]);
    const double mu = c.st.mu[p];
    if (!isfinite(lbh) || !isfinite(s) || !isfinite(mu)) v[5] += 1.0;
    v[1] += cj * (lbh - c.cols.logmarg[p]);
    v[2] += fabs(s - cj);
    v[3] += s * mu;
    v[4] += s;
  }
  block_reduce_store(v, 6, c.cert_part + (size_t)bx * 8);
}

__global__ __launch_bounds__(kBlock) void k_cert_partial(LaunchCtx c) { cert_partial_block(c, blockIdx.x, gridDim.x); }

__global__ __launch_bounds__(kBlock) void k_cert_partial_batch(const BatchItem* __restrict__ items,
                                                               const LaunchCtx* __restrict__ descs) {
  const BatchItem it = items[blockIdx.x];
  cert_partial_block(descs[it.prob], it.blk, descs[it.prob].cert_blocks);
}

__device__ __forceinline__ void cert_final_block(const LaunchCtx& c) {
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < c.cert_blocks; b += kBlock)
    for (int i = 0; i < 6; ++i) v[i] += c.cert_part[(size_t)b * 8 + i];
  __shared__ double tot[8];
  block_reduce_store(v, 6, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long k = c.ctrl->k - 1;  // the iteration just certified
    const double eps = c.ctrl->eta / (c.ctrl->lam * (double)k + 1.0);
    const double L = eps * (tot[0] + tot[1]);                 // <r, f> + <c, g>
    const double delta = 0.5 * tot[2];                        // 1/2 ||s - c||_1
    const double costZ = tot[3];                              // sum_j s_j mu_j
    const double U = costZ + c.ctrl->omega * delta;           // Algorithm 2
    double* o = c.cert_out;
    o[0] = (double)k;
    o[1] = eps;
    o[2] = L;
    o[3] = U;
    o[4] = delta;
    o[5] = costZ;
    o[6] = tot[4];
    o[7] = tot[5];
  }
}

__global__ __launch_bounds__(kBlock) void k_cert_final(LaunchCtx c) { cert_final_block(c); }

// one block per listed problem; also copies the record into a contiguous array
__global__ __launch_bounds__(kBlock) void k_cert_final_batch(const int* __restrict__ probs,
                                                             const LaunchCtx* __restrict__ descs,
                                                             double* __restrict__ records) {
  const LaunchCtx& c = descs[probs[blockIdx.x]];
  cert_final_block(c);
  __syncthreads();
  if (threadIdx.x < kCertSlots) {
    __threadfence_block();
    records[(size_t)blockIdx.x * kCertSlots + threadIdx.x] = c.cert_out[threadIdx.x];
  }
}

// repair: sum p, sum q, sum p|x|^2, sum q|y|^2, sum p x (3), sum q y (3), sum e s mu
__global__ __launch_bounds__(kBlock) void k_repair_partial(LaunchCtx c) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int stride = gridDim.x * kBlock;
  const int dim = c.dim;
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < c.rows.count; p += stride) {
    const double pv = c.st.pvec[p];
    double n2 = 0.0;
    for (int d = 0; d < dim; ++d) {
      const double xd = c.rows.abs[(size_t)d * c.rows.np + p];
      n2 += xd * xd;
      v[3 + d] += pv * xd;
    }
    v[0] += pv;
    v[2] += pv * n2;
  }
  block_reduce_store(v, 6, c.cert_part + (size_t)blockIdx.x * 8);
  __syncthreads();
  double w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < c.cols.count; p += stride) {
    const double s = exp(c.st.logs[p]);
    const double cj = c.cols.marg[p];
    const double q = cj > s ? cj - s : 0.0;
    const double e = cj < s ? cj / s : 1.0;
    double n2 = 0.0;
    for (int d = 0; d < dim; ++d) {
      const double yd = c.cols.abs[(size_t)d * c.cols.np + p];
      n2 += yd * yd;
      w[3 + d] += q * yd;
    }
    w[0] += q;
    w[1] += e * s * c.st.mu[p];
    w[2] += q * n2;
  }
  block_reduce_store(w, 6, c.cert_part + ((size_t)gridDim.x + blockIdx.x) * 8);
}

__global__ __launch_bounds__(kBlock) void k_repair_final(LaunchCtx c) {
  // partial layout: [0, G) row sums, [G, 2G) column sums
  double v[6] = {0, 0, 0, 0, 0, 0}, w[6] = {0, 0, 0, 0, 0, 0};
  const int G = c.cert_blocks;
  for (int b = threadIdx.x; b < G; b += kBlock)
    for (int i = 0; i < 6; ++i) {
      v[i] += c.cert_part[(size_t)b * 8 + i];
      w[i] += c.cert_part[(size_t)(G + b) * 8 + i];
    }
  __shared__ double tv[8], tw[8];
  block_reduce_store(v, 6, tv);
  __syncthreads();
  block_reduce_store(w, 6, tw);
  __syncthreads();
  if (threadIdx.x == 0) {
    // p^T C q = s [ (sum q)(sum p|x|^2) + (sum p)(sum q|y|^2) - 2 (sum p x).(sum q y) ]
    double cross = 0.0;
    for (int d = 0; d < c.dim; ++d) cross += tv[3 + d] * tw[3 + d];
    const double pCq = c.ctrl->scale * (tw[0] * tv[2] + tv[0] * tw[2] - 2.0 * cross);
    const double delta = c.cert_out[4];
    const double costClip = tw[1];                        // sum_j e_j s_j mu_j
    double* o = c.cert_out;
    o[8] = costClip + (delta > 0.0 ? pCq / delta : 0.0);   // <C, Z^>
    o[9] = tv[0];                                         // 1^T p
    o[10] = tw[0];                                        // 1^T q
    o[11] = pCq;
  }
}

// Rounded cost: sum_i cost_i + e_r^T C e_c / ||e_r||_1 with the squared
// Euclidean closed form e_r^T C e_c = s [ (sum e_c)(sum e_r |x|^2) +
// (sum e_r)(sum e_c |y|^2) - 2 (sum e_r x).(sum e_c y) ].  Row deficits in
// plan_aux, row costs in pvec, column deficits in mu (kFinishRound3 / 2).
__global__ __launch_bounds__(kBlock) void k_round_partial(LaunchCtx c) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int stride = gridDim.x * kBlock;
  const int dim = c.dim;
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < c.rows.count; p += stride) {
    const double er = c.plan_aux[p];
    double n2 = 0.0;
    for (int d = 0; d < dim; ++d) {
      const double xd = c.rows.abs[(size_t)d * c.rows.np + p];
      n2 += xd * xd;
      v[3 + d] += er * xd;
    }
    v[0] += er;
    v[1] += c.st.pvec[p];
    v[2] += er * n2;
  }
  block_reduce_store(v, 6, c.cert_part + (size_t)blockIdx.x * 8);
  __syncthreads();
  double w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < c.cols.count; p += stride) {
    const double ec = c.st.mu[p];
    double n2 = 0.0;
    for (int d = 0; d < dim; ++d) {
      const double yd = c.cols.abs[(size_t)d * c.cols.np + p];
      n2 += yd * yd;
      w[3 + d] += ec * yd;
    }
    w[0] += ec;
    w[2] += ec * n2;
  }
  block_reduce_store(w, 6, c.cert_part + ((size_t)gridDim.x + blockIdx.x) * 8);
}

__global__ __launch_bounds__(kBlock) void k_round_final(LaunchCtx c) {
  double v[6] = {0, 0, 0, 0, 0, 0}, w[6] = {0, 0, 0, 0, 0, 0};
  const int G = c.cert_blocks;
  for (int b = threadIdx.x; b < G; b += kBlock)
    for (int i = 0; i < 6; ++i) {
      v[i] += c.cert_part[(size_t)b * 8 + i];
      w[i] += c.cert_part[(size_t)(G + b) * 8 + i];
    }
  __shared__ double tv[8], tw[8];
  block_reduce_store(v, 6, tv);
  __syncthreads();
  block_reduce_store(w, 6, tw);
  __syncthreads();
  if (threadIdx.x == 0) {
    double dot = 0.0;
    for (int d = 0; d < c.dim; ++d) dot += tv[3 + d] * tw[3 + d];
    const double erCec = c.ctrl->scale * (tw[0] * tv[2] + tv[0] * tw[2] - 2.0 * dot);
    const double mass = tv[0];
    double* o = c.plan_stats;
    o[8] = tv[1] + (mass > 0.0 ? erCec / mass : 0.0);   // <C, G>
    o[9] = tv[1];                                       // <C, X''>
    o[10] = mass;                                       // ||e_r||_1
    o[11] = tw[0];                                      // ||e_c||_1 (equals ||e_r||_1)
  }
}

// Adds the per-wavefront tile counts of one sweep to the running total (one
// block, fixed order: profiling only).
__global__ __launch_bounds__(kBlock) void k_count_tiles(const unsigned* __restrict__ count, int n,
                                                        unsigned long long* __restrict__ total) {
  __shared__ unsigned long long part[kBlock];
  unsigned long long v = 0;
  for (int i = threadIdx.x; i < n; i += kBlock) v += count[i];
  part[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tsum = 0;
    for (int i = 0; i < kBlock; ++i) tsum += part[i];
    *total += tsum;
  }
}

__global__ void k_scatter(const double* __restrict__ src, const int* __restrict__ perm, int count,
                          double* __restrict__ dst) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p < count) dst[perm[p]] = src[p];
}

__global__ void k_hints_out(const int* __restrict__ hint, const int* __restrict__ perm_out,
                            const int* __restrict__ perm_in, int count, int* __restrict__ dst) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p < count) {
    const int j = hint[p];
    dst[perm_out[p]] = j >= 0 ? perm_in[j] : -1;
  }
}

__global__ void k_hints_in(const int* __restrict__ src, const int* __restrict__ perm_out,
                           const int* __restrict__ iperm_in, int count_in, int np, int* __restrict__ hint) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p < np) {
    const int j = src[perm_out[p]];
    hint[p] = (j >= 0 && j < count_in) ? iperm_in[j] : -1;
  }
}

__global__ void k_gather(const double* __restrict__ src, const int* __restrict__ perm, int np,
                         double* __restrict__ dst) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p < np) dst[p] = src[perm[p]];
}

// Factors of a feasible plan X_ij = exp(u_i + v_j - C_ij / eps) + a_i b_j, in
// original order.  Rounded state plan (Altschuler, Weed and Rigollet 2017,
// Algorithm 2): u = log alpha + log x, v = log beta + log y, a = e_r,
// b = e_c / ||e_r||_1.  Repaired intermediate plan (proof of Prop. 3):
// u = log alpha-hat, v = log t + log e with e_j = min(1, c_j / s_j), a = p,
// b = (c - s)_+ / delta.  lt_prev: log t of the last row update (repair only).
__global__ void k_export_factors(LaunchCtx c, int repaired, const double* __restrict__ lt_prev,
                                 double* __restrict__ u, double* __restrict__ v, double* __restrict__ a,
                                 double* __restrict__ b) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p < c.rows.count) {
    const int i = c.rows.perm[p];
    if (u) u[i] = repaired ? c.st.lah[p] : c.st.la[p] + c.plan_row[p];
    if (a) a[i] = repaired ? c.st.pvec[p] : c.plan_aux[p];
  }
  if (p < c.cols.count) {
    const int j = c.cols.perm[p];
    if (repaired) {
      const double ls = c.st.logs[p];
      const double delta = c.cert_out[4];
      if (v) v[j] = lt_prev[p] + fmin(0.0, c.cols.logmarg[p] - ls);
      if (b) b[j] = delta > 0.0 ? fmax(c.cols.marg[p] - exp(ls), 0.0) / delta : 0.0;
    } else {
      const double mass = c.plan_stats[10];
      if (v) v[j] = c.st.lb1[p] + c.plan_col[p];
      if (b) b[j] = mass > 0.0 ? c.st.mu[p] / mass : 0.0;
    }
  }
}

// Dense rows [row_begin, row_begin + nrows) of a factored plan, row-major in
// original order: out[(i - row_begin) n + j] = exp(u_i + v_j - kap |x_i - y_j|^2)
// (+ a_i b_j when R1), in float64 from the stored float32 coordinates.  One
// thread per column holds y_j, v_j and b_j.  A block walks strips of
// kEntryRows rows: its first wavefront loads the strip's slots, coordinates
// and factors (one lane per row, two round trips per strip) into LDS, and
// every thread then reads them from there for each row.  Write-bound: 8 bytes
// per entry.
constexpr int kEntryRows = 64;
template <int D, bool R1>
__global__ __launch_bounds__(kBlock) void k_plan_entries(LaunchCtx c, const double* __restrict__ u,
                                                         const double* __restrict__ v,
                                                         const double* __restrict__ a,
                                                         const double* __restrict__ b, double kap,
                                                         long long row_begin, long long nrows,
                                                         double* __restrict__ out) {
  __shared__ float sx[D][kEntryRows];
  __shared__ double su[kEntryRows], sa[kEntryRows];
  const int n = c.cols.count;
  const int j = blockIdx.y * kBlock + threadIdx.x;
  const bool col = j < n;  // no early return: every thread reaches the barriers
  double y[D];
  double vj = 0.0, bj = 0.0;
  if (col) {
    const int qj = c.cols.iperm[j];
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = (double)c.cols.abs[(size_t)d * c.cols.np + qj];
    vj = v[j];
    bj = R1 ? b[j] : 0.0;
  } else {
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = 0.0;
  }
  const long long blocks = (nrows + kEntryRows - 1) / kEntryRows;
  const long long last = row_begin + nrows - 1;
  for (long long rb = blockIdx.x; rb < blocks; rb += gridDim.x) {
    const long long r0 = rb * kEntryRows;
    const int rows = (int)min((long long)kEntryRows, nrows - r0);
    __syncthreads();  // the previous strip's rows have been read
    if (threadIdx.x < kEntryRows) {
      const long long i = min(row_begin + r0 + threadIdx.x, last);
      const int q = c.rows.iperm[i];
#pragma unroll
      for (int d = 0; d < D; ++d) sx[d][threadIdx.x] = c.rows.abs[(size_t)d * c.rows.np + q];
      su[threadIdx.x] = u[i];
      sa[threadIdx.x] = R1 ? a[i] : 0.0;
    }
    __syncthreads();
    if (!col) continue;
    double* o = out + (size_t)r0 * n + j;
    for (int t = 0; t < rows; ++t) {
      double d2 = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const double e = (double)sx[d][t] - y[d];
        d2 = fma(e, e, d2);
      }
      o[(size_t)t * n] = exp(su[t] + vj - kap * d2) + sa[t] * bj;
    }
  }
}

}  // namespace

hipError_t launch_sweep_batch(const BatchItem* items, int nitems, const LaunchCtx* descs, int dim,
                              bool transpose, bool cert, int kofs, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
#define BDRS_SWEEPB(DD, CC)                                                                       \
  hipLaunchKernelGGL((k_sweep_batch<DD, CC>), dim3(nitems), dim3(kSweepBlock), 0, s, items, descs,   \
                     transpose ? 1 : 0, kofs)
  switch (dim * 2 + (cert ? 1 : 0)) {
    case 2: BDRS_SWEEPB(1, kSweepPlain); break;
    case 3: BDRS_SWEEPB(1, kSweepCert); break;
    case 4: BDRS_SWEEPB(2, kSweepPlain); break;
    case 5: BDRS_SWEEPB(2, kSweepCert); break;
    case 6: BDRS_SWEEPB(3, kSweepPlain); break;
    case 7: BDRS_SWEEPB(3, kSweepCert); break;
    default: return hipErrorInvalidValue;
  }
#undef BDRS_SWEEPB
  return hipGetLastError();
}

hipError_t launch_finish_batch(const BatchItem* items, int nitems, const LaunchCtx* descs, bool transpose,
                               FinishKind kind, int kofs, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finish_batch, dim3(nitems), dim3(kTile), 0, s, items, descs, transpose ? 1 : 0,
                     (int)kind, kofs);
  return hipGetLastError();
}

hipError_t launch_advance(Ctrl* ctrl, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(kTile), 0, s, ctrl, n);
  return hipGetLastError();
}

hipError_t launch_advance_batch(const LaunchCtx* descs, int count, int n, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_advance_batch, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, descs, count, n);
  return hipGetLastError();
}

hipError_t launch_cert_batch(const BatchItem* items, int nitems, const int* probs, int nprobs,
                             const LaunchCtx* descs, double* records, hipStream_t s) {
  if (nitems <= 0 || nprobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cert_partial_batch, dim3(nitems), dim3(kBlock), 0, s, items, descs);
  hipLaunchKernelGGL(k_cert_final_batch, dim3(nprobs), dim3(kBlock), 0, s, probs, descs, records);
  return hipGetLastError();
}

int choose_splits(int np_out, int ntiles_in) {
  // enough (output wave, split) pairs to give every SIMD of the 256 CUs many
  // waves (skipped tiles make the work per pair uneven, so finer pairs balance
  // better), but at least 4 tiles per split so the per-split set-up stays
  // small; the partial records stay below target * 64 records plus one per
  // output
  const int out_waves = (np_out + kTile - 1) / kTile;
  int s = (BDRS_TARGET_WAVES + out_waves - 1) / out_waves;
  const int max_s = (ntiles_in + 3) / 4;
  if (s > max_s) s = max_s;
  if (s < 1) s = 1;
  const int tps = (ntiles_in + s - 1) / s;
  return (ntiles_in + tps - 1) / tps;  // splits that own at least one tile
}

hipError_t launch_sweep(const LaunchCtx& c, bool transpose, bool cert, int splits, double eps_arg, int kofs) {
  const SideDev& out = transpose ? c.cols : c.rows;
  const SideDev& in = transpose ? c.rows : c.cols;
  dim3 grid(splits, out.np / kSweepBlock);  // x: split, y: output block (see k_sweep)
#define BDRS_SWEEP(DD, CC)                                                                             \
  if (c.ev_start && c.ev_stop)                                                                         \
    hipExtLaunchKernelGGL((k_sweep<DD, CC>), grid, dim3(kSweepBlock), 0, c.stream, c.ev_start, c.ev_stop, \
                          0u, (const float*)out.abs, (int)out.np, (const float*)in.off,                 \
                          (const float*)in.A, (const TileRec*)in.tile, (int)in.ntiles, (int)in.count,   \
                          (int)splits, (const int*)out.hint, (void*)c.part.rec, (double*)c.part.ref, (const Ctrl*)c.ctrl, \
                          (double)eps_arg, (int)kofs, (int)(transpose ? 0 : 1), (unsigned*)c.tile_count);  \
  else                                                                                                 \
    hipLaunchKernelGGL((k_sweep<DD, CC>), grid, dim3(kSweepBlock), 0, c.stream, out.abs, out.np, in.off, \
                       in.A, in.tile, in.ntiles, in.count, splits, out.hint,                               \
                       c.part.rec, c.part.ref, c.ctrl, eps_arg, kofs, transpose ? 0 : 1, c.tile_count)
  switch (c.dim * 2 + (cert ? 1 : 0)) {
    case 2: BDRS_SWEEP(1, kSweepPlain); break;
    case 3: BDRS_SWEEP(1, kSweepCert); break;
    case 4: BDRS_SWEEP(2, kSweepPlain); break;
    case 5: BDRS_SWEEP(2, kSweepCert); break;
    case 6: BDRS_SWEEP(3, kSweepPlain); break;
    case 7: BDRS_SWEEP(3, kSweepCert); break;
    default: return hipErrorInvalidValue;
  }
#undef BDRS_SWEEP
  return hipGetLastError();
}

hipError_t launch_sweep_bary(const LaunchCtx& c, int splits, double eps) {
  const SideDev& out = c.rows;
  const SideDev& in = c.cols;
  dim3 grid(splits, out.np / kSweepBlock);  // x: split, y: output block (see k_sweep)
#define BDRS_SWEEP(DD)                                                                                  \
  hipLaunchKernelGGL((k_sweep<DD, kSweepBary>), grid, dim3(kSweepBlock), 0, c.stream, out.abs, out.np,   \
                     in.off, in.A, in.tile, in.ntiles, in.count, splits, out.hint, c.part.rec, c.part.ref, c.ctrl, eps, \
                     0, 1, \
                     c.tile_count)
  switch (c.dim) {
    case 1: BDRS_SWEEP(1); break;
    case 2: BDRS_SWEEP(2); break;
    case 3: BDRS_SWEEP(3); break;
    default: return hipErrorInvalidValue;
  }
#undef BDRS_SWEEP
  return hipGetLastError();
}

hipError_t launch_finish(const LaunchCtx& c, bool transpose, FinishKind kind, int splits, double eps_arg,
                         double* lse_out, int kofs) {
  // one wavefront per block (one tile of outputs), so the O(n) epilogue spreads over all CUs
  const SideDev& out = transpose ? c.cols : c.rows;
  hipLaunchKernelGGL(k_finish, dim3(out.ntiles), dim3(kTile), 0, c.stream, c, transpose ? 1 : 0,
                     (int)kind, splits, eps_arg, lse_out, kofs);
  return hipGetLastError();
}

hipError_t launch_prologue(const LaunchCtx& c) {
  hipLaunchKernelGGL(k_prologue, dim3(c.cols.np / kBlock), dim3(kBlock), 0, c.stream, c);
  return hipGetLastError();
}

hipError_t launch_pack(const LaunchCtx& c, bool transpose, const double* w, double eps) {
  const SideDev& in = transpose ? c.rows : c.cols;
  hipLaunchKernelGGL(k_pack, dim3(in.np / kBlock), dim3(kBlock), 0, c.stream, c, transpose ? 1 : 0, w, eps);
  return hipGetLastError();
}

hipError_t launch_pack_rows_from_lah(const LaunchCtx& c, double eps) {
  hipLaunchKernelGGL(k_pack_rows, dim3(c.rows.np / kBlock), dim3(kBlock), 0, c.stream, c, eps);
  return hipGetLastError();
}

hipError_t launch_count_tiles(const LaunchCtx& c, int n) {
  if (!c.tile_count || !c.tile_total || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_tiles, dim3(1), dim3(kBlock), 0, c.stream, c.tile_count, n, c.tile_total);
  return hipGetLastError();
}

hipError_t launch_pack_state(const LaunchCtx& c, bool transpose, double eps, bool with_factors) {
  const SideDev& in = transpose ? c.rows : c.cols;
  hipLaunchKernelGGL(k_pack_state, dim3(in.np / kBlock), dim3(kBlock), 0, c.stream, c, transpose ? 1 : 0, eps,
                     with_factors ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_round_reduce(const LaunchCtx& c) {
  // two sets of cert_blocks x 8 partials: the certificate's buffer holds both
  hipLaunchKernelGGL(k_round_partial, dim3(c.cert_blocks), dim3(kBlock), 0, c.stream, c);
  hipLaunchKernelGGL(k_round_final, dim3(1), dim3(kBlock), 0, c.stream, c);
  return hipGetLastError();
}

hipError_t launch_plan_stats(const LaunchCtx& c) {
  // the certificate's partial buffer holds cert_blocks x 8 doubles
  hipLaunchKernelGGL(k_plan_partial, dim3(c.cert_blocks), dim3(kBlock), 0, c.stream, c);
  hipLaunchKernelGGL(k_plan_final, dim3(1), dim3(kBlock), 0, c.stream, c, c.cert_blocks);
  return hipGetLastError();
}

hipError_t launch_cert_reduce(const LaunchCtx& c) {
  hipLaunchKernelGGL(k_cert_partial, dim3(c.cert_blocks), dim3(kBlock), 0, c.stream, c);
  hipLaunchKernelGGL(k_cert_final, dim3(1), dim3(kBlock), 0, c.stream, c);
  return hipGetLastError();
}

hipError_t launch_repair_pack(const LaunchCtx& c) {
  hipLaunchKernelGGL(k_repair_pack, dim3(c.cols.np / kBlock), dim3(kBlock), 0, c.stream, c);
  return hipGetLastError();
}

hipError_t launch_repair_reduce(const LaunchCtx& c) {
  hipLaunchKernelGGL(k_repair_partial, dim3(c.cert_blocks), dim3(kBlock), 0, c.stream, c);
  hipLaunchKernelGGL(k_repair_final, dim3(1), dim3(kBlock), 0, c.stream, c);
  return hipGetLastError();
}

hipError_t launch_export_factors(const LaunchCtx& c, bool repaired, const double* lt_prev, double* u, double* v,
                                 double* a, double* b) {
  const int cnt = std::max(c.rows.count, c.cols.count);
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_export_factors, dim3((cnt + kBlock - 1) / kBlock), dim3(kBlock), 0, c.stream, c,
                     repaired ? 1 : 0, lt_prev, u, v, a, b);
  return hipGetLastError();
}

hipError_t launch_plan_entries(const LaunchCtx& c, const double* u, const double* v, const double* a,
                               const double* b, double kap, long long row_begin, long long nrows, double* out) {
  if (nrows <= 0 || c.cols.count <= 0) return hipSuccess;
  const long long rblocks = (nrows + kEntryRows - 1) / kEntryRows;
  const dim3 grid((unsigned)std::min(rblocks, 65536LL), (unsigned)((c.cols.count + kBlock - 1) / kBlock));
#define BDRS_ENTRIES(DD, RR)                                                                        \
  hipLaunchKernelGGL((k_plan_entries<DD, RR>), grid, dim3(kBlock), 0, c.stream, c, u, v, a, b, kap, \
                     row_begin, nrows, out)
  const bool r1 = a != nullptr && b != nullptr;
  switch (c.dim * 2 + (r1 ? 1 : 0)) {
    case 2: BDRS_ENTRIES(1, false); break;
    case 3: BDRS_ENTRIES(1, true); break;
    case 4: BDRS_ENTRIES(2, false); break;
    case 5: BDRS_ENTRIES(2, true); break;
    case 6: BDRS_ENTRIES(3, false); break;
    default: BDRS_ENTRIES(3, true); break;
  }
#undef BDRS_ENTRIES
  return hipGetLastError();
}

hipError_t launch_scatter(const double* src, const int* perm, int count, double* dst, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, src, perm, count, dst);
  return hipGetLastError();
}

hipError_t launch_hints_out(const int* hint, const int* perm_out, const int* perm_in, int count, int* dst,
                            hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hints_out, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, hint, perm_out, perm_in,
                     count, dst);
  return hipGetLastError();
}

hipError_t launch_hints_in(const int* src, const int* perm_out, const int* iperm_in, int count_in, int np,
                           int* hint, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hints_in, dim3((np + kBlock - 1) / kBlock), dim3(kBlock), 0, s, src, perm_out, iperm_in,
                     count_in, np, hint);
  return hipGetLastError();
}

hipError_t launch_gather(const double* src, const int* perm, int np, double* dst, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((np + kBlock - 1) / kBlock), dim3(kBlock), 0, s, src, perm, np, dst);
  return hipGetLastError();
}

}  // namespace bdrs
