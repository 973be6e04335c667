// Internal declarations shared by the kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdrs {

constexpr int kTile = 64;         // points per tile = one wavefront
constexpr int kBlock = 256;       // threads per block of the O(n) kernels

// threads per sweep block: the waves of one block share the input tiles of
// their split (read once through the scalar cache for all of them)
#ifndef BDRS_SWEEP_BLOCK
#define BDRS_SWEEP_BLOCK 256
#endif
constexpr int kSweepBlock = BDRS_SWEEP_BLOCK;
constexpr int kPad = kSweepBlock > kBlock ? kSweepBlock : kBlock;  // np is a multiple of this
constexpr int kCertSlots = 16;    // doubles in a certificate record

// (output wavefront, split) pairs a sweep aims for: 4 per SIMD on 256 CUs
#ifndef BDRS_TARGET_WAVES
#define BDRS_TARGET_WAVES 16384
#endif

// Device-resident control block of one solver: the iteration counter lives
// here so that a captured block of iterations can be replayed at any k.
// Variant bits of Ctrl::variant (the same values as the public flags).
constexpr unsigned kVarOldKernel = 2u, kVarNoMomentum = 4u, kVarDebiased = 8u;
// Temperature standing in for the all-ones kernel K^{.0} of the old-kernel row
// update at k = 0: a factor 1e30 above eta makes every cost term vanish in
// float32 and float64 alike.
constexpr double kFarTemperature = 1e30;

struct Ctrl {
  long long k;             // first iteration of the current block of Algorithm 1
  unsigned int variant;    // ablation variant bits (0: Algorithm 1)
  unsigned int pad1;
  double eta, lam, scale;  // eta, lambda, cost scale s
  double omega;
};

// Everything the sweep needs to know about one input tile besides the offsets
// and weights of its points, read with a single 64-byte scalar load.
struct alignas(64) TileRec {
  double amax;    // tile maximum of w2 - kappa2 |b|^2 (float64; -inf: no mass)
  double alpha;   // intercept of the plane fit of the tile's log2 weights w2 over the
                  // offsets b: w2 <= alpha + gamma . b + rho for every point of the tile
  float ctr[3];   // tile centre (relative to the common origin)
  float rad[3];   // per-dimension radius of the offsets
  float gam[3];   // plane-fit gradient gamma
  float rho;      // largest residual of the fit, rounded up
  float pad[2];
};
static_assert(sizeof(TileRec) == 64, "one scalar dwordx16 load per tile");

// Geometry of one tile's real points, fixed for a solve: the epilogues fit a
// plane to the tile's log weights over these offsets, and with every real
// point live (the marginals are positive) the fit needs only the weighted
// sums.  cinv holds the inverse of the centred scatter matrix sum (b - mb)
// (b - mb)^T (entries xx, xy, xz, yy, yz, zz; all 0 when it is near singular:
// then the plane is flat).
struct TileGeom {
  double mb[3];    // mean offset of the real points
  double cinv[6];
  double cnt;      // real points
};

// One point set stored in tile order.  Slot p holds original point perm[p];
// slots >= count are padding (copies of a real point with weight -inf).
struct SideDev {
  int count;       // real points
  int ntiles;      // ceil(count / 64)
  int np;          // ntiles * 64, padded to a multiple of 256 for the epilogues
  int pad;
  float* abs;      // [dim][np] coordinates relative to the common origin (SoA)
  float* off;      // [ntiles][dim][64] offsets from the tile centre
  float* A;        // [np] log2 weights of the next sweep that reads this side minus their
                   //      tile's plane fit and the tile-local quadratic (float32)
  TileRec* tile;   // [ntiles] per-tile record (maximum, plane fit, centre, radius)
  const TileGeom* geom;  // [ntiles] geometry of the real points
  int* perm;       // [np] original index of each slot
  int* iperm;      // [count] slot of each original index
  int* hint;       // [np] warm start of the sweep with this side as output: the slot of an
                   //      input point whose term is near the output's maximum, or -1
  double* marg;    // [np] marginal (r or c), 0 on padding
  double* logmarg; // [np] log marginal
};

// Dual state (float64, tile order; O(m + n)).
struct StateDev {
  double* la;       // log alpha^{k-1}  (rows)
  double* lah;      // log alpha-hat    (rows)
  double* lb1;      // log beta^{k-1}   (cols)
  double* lb2;      // log beta^{k-2}   (cols)
  double* lbh;      // log beta-hat     (cols)
  double* lt[2];    // log beta-tilde, ping-pong by parity of k (cols)
  double* mu;       // certificate: mean column cost mu_j
  double* logs;     // certificate: log s_j
  double* pvec;     // repair: row deficits p_i
};

// Partial reduction of one (split, output) of a sweep.  dM is the split's
// shift (log2) relative to the output's reference R (the exponent of its warm
// start, the same in every split; 0 when there is none), kept in float32: the
// sweep rescales its shifted sums by the rounding of dM, so that S 2^{R + dM}
// is the split's sum to float32 accuracy.  S: shifted sum; J: input slot of
// the term that set the shift (the warm start's unless an exact-max pass
// raised it; -1 for none).  12 bytes; R is stored once per output.
struct PartialRec {
  float dM;
  float S;
  int J;
};
// The same for certificate sweeps, with the shifted cost-weighted sum N
// (Algorithm 2's column statistics).  16 bytes.
struct PartialCert {
  float dM;
  float S;
  float N;
  int J;
};

// Partial of the barycentric sweep: shift M (float64), shifted sum S and the
// shifted sum of the input points' coordinates V.  24 bytes.
struct PartialBary {
  double M;
  float S;
  float V[3];
};
// bytes per (split, output) slot of the partial buffer: the largest record
constexpr int kPartialSlot = 24;
static_assert(sizeof(PartialRec) <= kPartialSlot && sizeof(PartialCert) <= kPartialSlot &&
                  sizeof(PartialBary) <= kPartialSlot, "every partial fits a slot");

// What a sweep accumulates besides the shifted sum.
enum SweepMode {
  kSweepPlain = 0,
  kSweepCert = 1,   // cost-weighted sum (Algorithm 2's N_j)
  kSweepBary = 2    // coordinate-weighted sums (barycentric projection)
};

struct Partials {
  void* rec;        // [S][np] records of the sweep's mode (PartialRec, PartialCert or PartialBary)
  double* ref;      // [np] per-output reference R of the records (largest np of the two sides)
  int splits;       // allocated splits
};

enum FinishKind {
  kFinishRow = 0,       // Algorithm 1 row epilogue
  kFinishCol = 1,       // Algorithm 1 column epilogue (advances k)
  kFinishColCert = 2,   // column epilogue + Algorithm 2 column statistics
  kFinishLse = 3,       // plain LSE output (parity entry point)
  kFinishRepair = 4,    // repair deficits p_i
  kFinishCertOnly = 5,  // Algorithm 2 column statistics of the last finished iteration
  kFinishPlanRow = 6,   // state plan: row sums and barycentric projection (bary partials)
  kFinishPlanCol = 7,   // state plan: column sums
  kFinishRound1 = 8,    // rounding: row factors x = min(1, r / X 1)
  kFinishRound2 = 9,    // rounding: column factors y = min(1, c / X'^T 1) and column deficits
  kFinishRound3 = 10    // rounding: row deficits and the cost of the scaled plan (cert partials)
};

struct LaunchCtx {
  hipStream_t stream;
  int dim;
  int splits_row, splits_col;  // input splits of the row / column sweep
  Ctrl* ctrl;
  SideDev rows, cols;
  StateDev st;
  Partials part;
  double* cert_part;   // [cert_blocks][8]
  double* cert_out;    // [kCertSlots]
  int cert_blocks;
  double* plan_row;    // [rows.np] row sums of the state plan (tile order)
  double* plan_col;    // [cols.np] column sums of the state plan (tile order)
  double* plan_aux;    // [rows.np] the rounding's row deficits e_r (tile order)
  double* plan_stats;  // [kCertSlots] marginal-error statistics
  double origin[3];    // common origin of the stored coordinates
  // profiling only (null otherwise): one slot per sweep wavefront receiving
  // the number of input tiles it evaluated, and their running total
  unsigned* tile_count;
  unsigned long long* tile_total;
  // profiling only (null otherwise): events the sweep launch itself records at
  // the start and the end of the kernel (not around its dispatch)
  hipEvent_t ev_start, ev_stop;
};

// One work item of a batched phase: problem index into the descriptor array,
// block of outputs (or output tile), and input split (sweeps only).
struct BatchItem {
  int prob, blk, split, pad;
};

// Kernel launchers (bdrs_kernels.hip).  Each returns the launch status.
// kofs: offset of the iteration inside the current block (k = Ctrl::k + kofs);
// launch_advance adds a finished block's length to Ctrl::k.
// An iteration's sweeps (eps_arg <= 0) take the row update's temperature when
// the rows are the outputs and the column update's otherwise.
hipError_t launch_sweep(const LaunchCtx& c, bool transpose, bool cert, int splits, double eps_arg, int kofs);
hipError_t launch_finish(const LaunchCtx& c, bool transpose, FinishKind kind, int splits,
                         double eps_arg, double* lse_out, int kofs);
hipError_t launch_advance(Ctrl* ctrl, int n, hipStream_t s);
hipError_t launch_prologue(const LaunchCtx& c);                       // lt and A_C for iteration k
hipError_t launch_pack(const LaunchCtx& c, bool transpose, const double* w, double eps);
hipError_t launch_pack_rows_from_lah(const LaunchCtx& c, double eps);
// state plan: input side packed from the state (columns: log beta, rows: log alpha),
// plus the rounding's log factors (plan_col / plan_row) when with_factors
hipError_t launch_pack_state(const LaunchCtx& c, bool transpose, double eps, bool with_factors = false);
hipError_t launch_round_reduce(const LaunchCtx& c);
// row sweep accumulating the input coordinates (barycentric projection)
hipError_t launch_sweep_bary(const LaunchCtx& c, int splits, double eps);
// adds the per-wavefront tile counts of the last sweep (n slots) to *tile_total
hipError_t launch_count_tiles(const LaunchCtx& c, int n);
hipError_t launch_plan_stats(const LaunchCtx& c);
hipError_t launch_cert_reduce(const LaunchCtx& c);
hipError_t launch_repair_pack(const LaunchCtx& c);
hipError_t launch_repair_reduce(const LaunchCtx& c);
// factors of the rounded (repaired = false) or repaired plan in original order;
// null outputs are skipped
hipError_t launch_export_factors(const LaunchCtx& c, bool repaired, const double* lt_prev, double* u, double* v,
                                 double* a, double* b);
// dense rows [row_begin, row_begin + nrows) of a factored plan (kap = cost scale / eps)
hipError_t launch_plan_entries(const LaunchCtx& c, const double* u, const double* v, const double* a,
                               const double* b, double kap, long long row_begin, long long nrows, double* out);
hipError_t launch_scatter(const double* src, const int* perm, int count, double* dst, hipStream_t s);
hipError_t launch_gather(const double* src, const int* perm, int np, double* dst, hipStream_t s);
// hints: to original order (out[perm_out[p]] = perm_in[hint[p]]) and back
hipError_t launch_hints_out(const int* hint, const int* perm_out, const int* perm_in, int count, int* dst,
                            hipStream_t s);
hipError_t launch_hints_in(const int* src, const int* perm_out, const int* iperm_in, int count_in, int np,
                           int* hint, hipStream_t s);

// Batched phases over the problems in `descs` (device array of LaunchCtx).
hipError_t launch_sweep_batch(const BatchItem* items, int nitems, const LaunchCtx* descs, int dim,
                              bool transpose, bool cert, int kofs, hipStream_t s);
hipError_t launch_finish_batch(const BatchItem* items, int nitems, const LaunchCtx* descs, bool transpose,
                               FinishKind kind, int kofs, hipStream_t s);
hipError_t launch_advance_batch(const LaunchCtx* descs, int count, int n, hipStream_t s);
hipError_t launch_cert_batch(const BatchItem* items, int nitems, const int* probs, int nprobs,
                             const LaunchCtx* descs, double* records, hipStream_t s);

int choose_splits(int np_out, int ntiles_in);

}  // namespace bdrs
