// gfx950 kernels of the Dual O-BDRS hot path.
//
// Sweep (the reduction of Algorithm 1's row and column updates, and of
// Algorithm 2's column pass).  For every output point p of one side and the
// input points q of the other side it evaluates, in base 2,
//     LSE2_p = log2 sum_q 2^{ w2_q - kappa2 ||P_p - Q_q||^2 },
//     kappa2 = log2(e) * s / eps,   w2 = log2(e) * w,
// which is LSE_q(w_q - C_pq / eps) / ln 2.  The cost is never stored: inputs
// are grouped in tiles of 64 spatially close points with centre Qc, offsets
// b_q = Q_q - Qc, and with a = P_p - Qc the exponent expands exactly as
//     w2_q - kappa2 |a - b_q|^2 = A_q + (2 kappa2 a) . b_q - kappa2 |a|^2,
//     A_q = w2_q - kappa2 |b_q|^2   (written by the producing epilogue),
// i.e. d FMAs and one add per entry, then one v_exp_f32 and one add.
//
// Precision split.  The weights w grow like g / eps as the temperature falls,
// so float32 values of that size would carry absolute errors u |g| / eps.  The
// inner loop therefore only sees small numbers: A_q is stored relative to its
// tile maximum, A'_q = A_q - Amax_t (float32), and the large per-(output, tile)
// part base = Amax_t - kappa2 |a|^2 and the lane's running shift M are kept in
// float64.  The summand is 2^{cm + B . b_q + A'_q} with cm = base - M (float32,
// small for the tiles that dominate the sum).
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

#include <math.h>

namespace bdrs {

namespace {

constexpr double kLog2eD = 1.4426950408889634074;
constexpr double kLn2D = 0.69314718055994530942;
constexpr float kThresh = 64.0f;

template <typename CtrlPtr>
__device__ __forceinline__ double eps_of(CtrlPtr c, double eps_arg, int kshift) {
  if (eps_arg > 0.0) return eps_arg;
  return c->eta / (c->lam * (double)(c->k + kshift) + 1.0);  // eta_k = eta / (lambda k + 1)
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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

// One block of 256 outputs (bx) against one split of the input tiles.
template <int D, bool CERT>
__device__ __forceinline__ void sweep_block(
    gfloat* __restrict__ out_abs, int np_out,
    gfloat* __restrict__ in_off, gfloat* __restrict__ in_hdr,
    gfloat* __restrict__ in_A, gdouble* __restrict__ in_Amax,
    int ntiles_in, int tps,
    PartialRec* __restrict__ part, gctrl* __restrict__ ctrl, double eps_arg, int bx, int split) {
  const int p = bx * kBlock + threadIdx.x;
  const int t0 = split * tps;
  const int t1 = min(t0 + tps, ntiles_in);
  const double eps = eps_of(ctrl, eps_arg, 0);
  const double kap2d = kLog2eD * ctrl->scale / eps;
  const float kap2x2 = (float)(2.0 * kap2d);

  float P[D];
#pragma unroll
  for (int d = 0; d < D; ++d) P[d] = out_abs[(size_t)d * np_out + p];

  double M = -INFINITY;
  float S = 0.0f, N = 0.0f;

  for (int t = t0; t < t1; ++t) {
    gfloat* __restrict__ hdr = in_hdr + (size_t)t * kHdr;
    const double amax = in_Amax[t];
    if (amax == -INFINITY) continue;  // tile carries no mass (masked weights)
    float a[D], B[D], na = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      a[d] = P[d] - hdr[d];
      na = fmaf(a[d], a[d], na);
      B[d] = kap2x2 * a[d];
    }
    const double base = amax - kap2d * (double)na;  // Amax_t - kappa2 |a|^2
    float bnd = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) bnd = fmaf(fabsf(B[d]), hdr[3 + d], bnd);

    gfloat* __restrict__ offs = in_off + (size_t)t * D * kTile;
    gfloat* __restrict__ Aq = in_A + (size_t)t * kTile;

    if (base + (double)bnd > M + kThresh) {
      // exact maximum of this tile for the lanes whose bound exceeds the window
      float tm = -INFINITY;
#pragma unroll 16
      for (int q = 0; q < kTile; ++q) {
        float z = Aq[q];
#pragma unroll
        for (int d = 0; d < D; ++d) z = fmaf(B[d], offs[d * kTile + q], z);
        tm = fmaxf(tm, z);
      }
      const double tmd = base + (double)tm;
      if (tmd > M) {
        const float sc = fast_exp2((float)(M - tmd));
        S *= sc;
        if (CERT) N *= sc;
        M = tmd;
      }
    }
    const float cm = (float)(base - M);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    float n0 = 0.f, n1 = 0.f;
#pragma unroll 16
    for (int q = 0; q < kTile; q += 4) {
      float e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float z = cm;
#pragma unroll
        for (int d = 0; d < D; ++d) z = fmaf(B[d], offs[d * kTile + q + u], z);
        z += Aq[q + u];
        e[u] = fast_exp2(z);
        if (CERT) {
          float c2 = 0.0f;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const float df = a[d] - offs[d * kTile + q + u];
            c2 = fmaf(df, df, c2);
          }
          if (u & 1) n1 = fmaf(c2, e[u], n1); else n0 = fmaf(c2, e[u], n0);
        }
      }
      s0 += e[0];
      s1 += e[1];
      s2 += e[2];
      s3 += e[3];
    }
    S += (s0 + s1) + (s2 + s3);
    if (CERT) N += n0 + n1;
  }
  PartialRec rec;
  rec.M = M;
  rec.S = S;
  rec.N = CERT ? N : 0.0f;
  part[(size_t)split * np_out + p] = rec;
}

template <int D, bool CERT>
__global__ __launch_bounds__(kBlock) void k_sweep(
    const float* __restrict__ out_abs, int np_out,
    const float* __restrict__ in_off, const float* __restrict__ in_hdr,
    const float* __restrict__ in_A, const double* __restrict__ in_Amax,
    int ntiles_in, int tps,
    PartialRec* __restrict__ part, const Ctrl* __restrict__ ctrl, double eps_arg) {
  sweep_block<D, CERT>((gfloat*)out_abs, np_out, (gfloat*)in_off, (gfloat*)in_hdr, (gfloat*)in_A,
                       (gdouble*)in_Amax, ntiles_in, tps, part, (gctrl*)ctrl, eps_arg, blockIdx.x,
                       blockIdx.y);
}

// Batched sweep: block i runs work item i = (problem, block of outputs, split)
// of a list over several problems; the arithmetic per item is the same as in
// the single-problem launch.
template <int D, bool CERT>
__global__ __launch_bounds__(kBlock) void k_sweep_batch(const BatchItem* __restrict__ items,
                                                        const LaunchCtx* __restrict__ descs, int transpose) {
  const BatchItem it = items[blockIdx.x];
  const LaunchCtx& c = descs[it.prob];
  const SideDev& out = transpose ? c.cols : c.rows;
  const SideDev& in = transpose ? c.rows : c.cols;
  const int splits = transpose ? c.splits_col : c.splits_row;
  const int tps = (in.ntiles + splits - 1) / splits;
  sweep_block<D, CERT>((gfloat*)out.abs, out.np, (gfloat*)in.off, (gfloat*)in.hdr, (gfloat*)in.A,
                       (gdouble*)in.Amax, in.ntiles, tps, c.part.rec, (gctrl*)c.ctrl, -1.0, it.blk,
                       it.split);
}

// ---------------------------------------------------------------------------
// Finish: merge the split partials (float64) and run the epilogue.
// ---------------------------------------------------------------------------
struct Merged {
  double lse;   // natural-log LSE
  double S;     // merged shifted sum (relative to Mx)
  double N;     // merged shifted cost sum
};

__device__ __forceinline__ Merged merge_splits(const PartialRec* __restrict__ part, int splits, int np,
                                               int p) {
  // all loads of a group of 8 splits are issued before they are used
  constexpr int G = 8;
  double mx = -INFINITY;
  for (int s0 = 0; s0 < splits; s0 += G) {
    double m[G];
#pragma unroll
    for (int g = 0; g < G; ++g) m[g] = (s0 + g < splits) ? part[(size_t)(s0 + g) * np + p].M : -INFINITY;
#pragma unroll
    for (int g = 0; g < G; ++g) mx = fmax(mx, m[g]);
  }
  Merged r{-INFINITY, 0.0, 0.0};
  if (mx == -INFINITY) return r;  // empty sum
  double S = 0.0, N = 0.0;
  for (int s0 = 0; s0 < splits; s0 += G) {
    PartialRec q[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (s0 + g < splits) q[g] = part[(size_t)(s0 + g) * np + p];
      else q[g] = PartialRec{-INFINITY, 0.0f, 0.0f};
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      // shifts of one output differ by little: the weight is a hardware float32 exp2
      const double w = (double)fast_exp2((float)(q[g].M - mx));  // 0 for an empty split
      S += w * (double)q[g].S;
      N += w * (double)q[g].N;
    }
  }
  r.S = S;
  r.N = N;
  r.lse = kLn2D * (mx + log2(S));
  return r;
}

__device__ __forceinline__ float norm2_off(const float* __restrict__ off, int dim, int p) {
  const int t = p / kTile, q = p % kTile;
  float s = 0.0f;
  for (int d = 0; d < dim; ++d) {
    const float b = off[((size_t)t * dim + d) * kTile + q];
    s = fmaf(b, b, s);
  }
  return s;
}

// A_p = log2(e) w - kappa2 |b_p|^2 in float64 (-inf on padding or for w = -inf);
// stores the tile maximum (float64) and A_p minus that maximum (float32).
// Called by whole wavefronts (one tile per wavefront).
__device__ __forceinline__ void pack_weight(const SideDev& sd, int dim, int p, double w, double kap2) {
  double A = -INFINITY;
  if (p < sd.count && w > -INFINITY) A = kLog2eD * w - kap2 * (double)norm2_off(sd.off, dim, p);
  if (p < sd.ntiles * kTile) {
    const double m = wave_max(A);
    sd.A[p] = (A == -INFINITY) ? -INFINITY : (float)(A - m);
    if ((threadIdx.x & (kTile - 1)) == 0) sd.Amax[p / kTile] = m;
  }
}

// Merge + epilogue of one tile (bx) of 64 outputs; nblocks = tiles of the
// output side (the column epilogue's last block advances k).
__device__ __forceinline__ void finish_block(const LaunchCtx& c, int transpose, int kind, int splits,
                                             double eps_arg, double* __restrict__ lse_out, int bx,
                                             int nblocks) {
  const SideDev& out = transpose ? c.cols : c.rows;
  const int p = bx * kTile + threadIdx.x;
  const int np = out.np;
  if (p >= np) return;
  const bool cert = (kind == kFinishColCert || kind == kFinishCertOnly);
  const Merged mg = merge_splits(c.part.rec, splits, np, p);
  const bool real = p < out.count;
  const Ctrl* ctrl = c.ctrl;
  const long long k = ctrl->k;
  const double lam = ctrl->lam;

  if (kind == kFinishLse) {
    if (real) lse_out[out.perm[p]] = mg.lse;
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
    // Algorithm 1: log alpha-hat^k = log r - LSE, log alpha^k = (1-lambda) log alpha^{k-1} + lambda log alpha-hat^k
    const double eps = eps_of(ctrl, eps_arg, 0);
    const double kap2 = kLog2eD * ctrl->scale / eps;
    double lah = 0.0;
    if (real) {
      lah = out.logmarg[p] - mg.lse;
      c.st.lah[p] = lah;
      c.st.la[p] = (1.0 - lam) * c.st.la[p] + lam * lah;
    }
    // weights of the column sweep of the same iteration: w = log alpha-hat
    pack_weight(c.rows, c.dim, p, lah, kap2);
    return;
  }
  // column epilogue (plain or certificate)
  const int cur = (int)(k & 1), nxt = (int)((k + 1) & 1);
  if (real) {
    const double lbh = out.logmarg[p] - mg.lse;         // log beta-hat^k = log c - LSE
    const double lb1 = c.st.lb1[p];
    const double lb = (1.0 - lam) * lb1 + lam * lbh;    // log beta^k
    if (cert) {
      // Algorithm 2: mu_j = N_j / D_j, d_j = M_j + log D_j, log s_j = log t_j + d_j
      c.st.mu[p] = ctrl->scale * mg.N / mg.S;
      c.st.logs[p] = c.st.lt[cur][p] + mg.lse;
    }
    c.st.lbh[p] = lbh;
    c.st.lb2[p] = lb1;
    c.st.lb1[p] = lb;
    // momentum for iteration k+1: log beta-tilde^k = log beta^k + (log beta^k - log beta^{k-1}) / lambda
    c.st.lt[nxt][p] = lb + (lb - lb1) / lam;
  }
  const double eps1 = eps_of(ctrl, -1.0, 1);
  const double kap2n = kLog2eD * ctrl->scale / eps1;
  pack_weight(c.cols, c.dim, p, real ? c.st.lt[nxt][p] : 0.0, kap2n);

  // the last block to finish advances k: every block read k at its start and
  // used it before counting itself here, and the next kernel sees the store
  if (threadIdx.x == 0) {
    const unsigned int done = atomicAdd(&c.ctrl->arrive, 1u);
    if (done == (unsigned int)nblocks - 1) {
      c.ctrl->arrive = 0u;
      c.ctrl->k = k + 1;
    }
  }
}

__global__ __launch_bounds__(kTile) void k_finish(LaunchCtx c, int transpose, int kind, int splits,
                                                  double eps_arg, double* __restrict__ lse_out) {
  finish_block(c, transpose, kind, splits, eps_arg, lse_out, blockIdx.x, gridDim.x);
}

// Batched merge + epilogue: block i runs item i = (problem, output tile).
__global__ __launch_bounds__(kTile) void k_finish_batch(const BatchItem* __restrict__ items,
                                                        const LaunchCtx* __restrict__ descs, int transpose,
                                                        int kind) {
  const BatchItem it = items[blockIdx.x];
  const LaunchCtx& c = descs[it.prob];
  const SideDev& out = transpose ? c.cols : c.rows;
  finish_block(c, transpose, kind, transpose ? c.splits_col : c.splits_row, -1.0, nullptr, it.blk, out.ntiles);
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
    lt = lb1 + (lb1 - lb2) / lam;
    c.st.lt[k & 1][p] = lt;
  }
  const double kap2 = kLog2eD * c.ctrl->scale / eps_of(c.ctrl, -1.0, 0);
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
  const double kap2 = kLog2eD * c.ctrl->scale / eps_of(c.ctrl, -1.0, -1);
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
  for (int p = bx * kBlock + threadIdx.x; p < c.rows.count; p += stride) {
    const double lah = c.st.lah[p];
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

__global__ void k_scatter(const double* __restrict__ src, const int* __restrict__ perm, int count,
                          double* __restrict__ dst) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p < count) dst[perm[p]] = src[p];
}

__global__ void k_gather(const double* __restrict__ src, const int* __restrict__ perm, int np,
                         double* __restrict__ dst) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p < np) dst[p] = src[perm[p]];
}

}  // namespace

hipError_t launch_sweep_batch(const BatchItem* items, int nitems, const LaunchCtx* descs, int dim,
                              bool transpose, bool cert, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
#define BDRS_SWEEPB(DD, CC)                                                                       \
  hipLaunchKernelGGL((k_sweep_batch<DD, CC>), dim3(nitems), dim3(kBlock), 0, s, items, descs,   \
                     transpose ? 1 : 0)
  switch (dim * 2 + (cert ? 1 : 0)) {
    case 2: BDRS_SWEEPB(1, false); break;
    case 3: BDRS_SWEEPB(1, true); break;
    case 4: BDRS_SWEEPB(2, false); break;
    case 5: BDRS_SWEEPB(2, true); break;
    case 6: BDRS_SWEEPB(3, false); break;
    case 7: BDRS_SWEEPB(3, true); break;
    default: return hipErrorInvalidValue;
  }
#undef BDRS_SWEEPB
  return hipGetLastError();
}

hipError_t launch_finish_batch(const BatchItem* items, int nitems, const LaunchCtx* descs, bool transpose,
                               FinishKind kind, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finish_batch, dim3(nitems), dim3(kTile), 0, s, items, descs, transpose ? 1 : 0,
                     (int)kind);
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
  // enough (output wave, split) pairs to give every SIMD of the 256 CUs a few
  // waves, but at least 4 tiles per split so the per-split set-up stays small
  const int out_waves = (np_out + kTile - 1) / kTile;
  int s = (BDRS_TARGET_WAVES + out_waves - 1) / out_waves;
  const int max_s = (ntiles_in + 3) / 4;
  if (s > max_s) s = max_s;
  if (s < 1) s = 1;
  const int tps = (ntiles_in + s - 1) / s;
  return (ntiles_in + tps - 1) / tps;  // splits that own at least one tile
}

hipError_t launch_sweep(const LaunchCtx& c, bool transpose, bool cert, int splits, double eps_arg) {
  const SideDev& out = transpose ? c.cols : c.rows;
  const SideDev& in = transpose ? c.rows : c.cols;
  const int tps = (in.ntiles + splits - 1) / splits;
  dim3 grid(out.np / kBlock, splits);
#define BDRS_SWEEP(DD, CC)                                                                          \
  hipLaunchKernelGGL((k_sweep<DD, CC>), grid, dim3(kBlock), 0, c.stream, out.abs, out.np, in.off,  \
                     in.hdr, in.A, in.Amax, in.ntiles, tps, c.part.rec, c.ctrl, eps_arg)
  switch (c.dim * 2 + (cert ? 1 : 0)) {
    case 2: BDRS_SWEEP(1, false); break;
    case 3: BDRS_SWEEP(1, true); break;
    case 4: BDRS_SWEEP(2, false); break;
    case 5: BDRS_SWEEP(2, true); break;
    case 6: BDRS_SWEEP(3, false); break;
    case 7: BDRS_SWEEP(3, true); break;
    default: return hipErrorInvalidValue;
  }
#undef BDRS_SWEEP
  return hipGetLastError();
}

hipError_t launch_finish(const LaunchCtx& c, bool transpose, FinishKind kind, int splits, double eps_arg,
                         double* lse_out) {
  // one wavefront per block (one tile of outputs), so the O(n) epilogue spreads over all CUs
  const SideDev& out = transpose ? c.cols : c.rows;
  hipLaunchKernelGGL(k_finish, dim3(out.ntiles), dim3(kTile), 0, c.stream, c, transpose ? 1 : 0,
                     (int)kind, splits, eps_arg, lse_out);
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

hipError_t launch_scatter(const double* src, const int* perm, int count, double* dst, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, src, perm, count, dst);
  return hipGetLastError();
}

hipError_t launch_gather(const double* src, const int* perm, int np, double* dst, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((np + kBlock - 1) / kBlock), dim3(kBlock), 0, s, src, perm, np, dst);
  return hipGetLastError();
}

}  // namespace bdrs
