// Internal declarations of the host runtime (shared by the C ABI, the batch
// engine and the solve server).
#pragma once
#include "bdrs_internal.h"
#include "../../include/bdrs.h"

#include <string>
#include <vector>

namespace bdrs_host {

using namespace bdrs;

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bdrs_status fail(bdrs_status st, const char* fmt, ...);
bdrs_status hip_status(hipError_t e, const char* what);

struct SideShape {
  int count, ntiles, np;
};

// Offsets of every sub-buffer inside the workspace.
struct Layout {
  SideShape R, C;
  int splits_row, splits_col, splits_max;
  int cert_blocks;
  size_t total;
  // offsets
  size_t ctrl;
  size_t r_abs, r_off, r_tile, r_geom, r_A, r_perm, r_marg, r_logm, r_iperm, r_hint;
  size_t c_abs, c_off, c_tile, c_geom, c_A, c_perm, c_marg, c_logm, c_iperm, c_hint;
  size_t la, lah, lb1, lb2, lbh, lt0, lt1, mu, logs, pvec;
  size_t part, part_ref, cert_part, cert_out, plan_row, plan_col, plan_aux, plan_stats, tile_count, tile_total;
  // retained best state (BDRS_F_KEEP_BEST_STATE; 0 otherwise), in tile order
  bool keep_best;
  size_t best_la, best_lah, best_lb1, best_lb2, best_lbh, best_lt0, best_lt1, best_hr, best_hc;
};

// Split counts of the tuning table for this shape, if it holds an entry.
bool tuned_splits(int dim, int m, int n, int* splits_row, int* splits_col);
// A split count clamped to [1, ntiles_in] and reduced to the number of splits
// that own at least one input tile at ceil(ntiles_in / s) tiles per split.
int normalize_splits(int s, int ntiles_in);
// Workspace layout; the partial records get room for at least reserve_row /
// reserve_col splits (the autotuner's largest candidates).
Layout make_layout(int m, int n, int dim, int reserve_row = 0, int reserve_col = 0, bool keep_best = false);
bdrs_status check_sizes(const bdrs_params* p);
// need = 0: the workspace must hold make_layout(m, n, dim)
bdrs_status check_params(const bdrs_params* p, size_t need = 0);
bdrs_status check_device();

// One point set in tile order on the host: what bdrs_create uploads for it.
struct HostSide {
  std::vector<float> abs, off;
  std::vector<TileRec> tile;
  std::vector<TileGeom> geom;
  std::vector<int> perm, iperm;
  std::vector<double> marg, logm;
};

// A problem prepared on the host (contents validated, points in Morton tile
// order, tile records and offsets built); independent of the split counts.
struct HostImage {
  int m = 0, n = 0, dim = 0;
  double origin[3] = {0, 0, 0};
  HostSide R, C;
};

// Validates the contents of host copies of the inputs and builds the image.
bdrs_status prepare_image(const bdrs_params* p, const float* hx, const float* hy, const double* hr,
                          const double* hc, HostImage& img);
// Lays out the workspace, uploads the image, initialises the state of
// Algorithm 1 (synchronises p->stream).
bdrs_status create_from_image(const bdrs_params* p, const HostImage& img, bdrs_solver* out, int reserve_row = 0,
                              int reserve_col = 0);
// Both steps: a solver from host copies of the inputs.
bdrs_status create_from_host(const bdrs_params* p, const float* hx, const float* hy, const double* hr,
                             const double* hc, bdrs_solver* out, int reserve_row = 0, int reserve_col = 0);
// Device -> host copies of a problem's inputs (synchronises p->stream).
bdrs_status download_inputs(const bdrs_params* p, std::vector<float>& hx, std::vector<float>& hy,
                            std::vector<double>& hr, std::vector<double>& hc);
bdrs_status hip_status(hipError_t e, const char* what);
bdrs_status sync_k(bdrs_solver s);
bdrs_status cert_from_record(bdrs_solver s, const double* rec, bool repair, bdrs_cert* out);

struct BatchLayout {
  size_t descs, items_rs, items_cs, items_rf, items_cf, items_ce, probs, records, total;
  size_t n_rs, n_cs, n_rf, n_cf, n_ce;  // item capacities (all problems active)
};

// Runs blocks of iterations for a set of solvers (same dim) with one launch
// per phase over work lists of all members.  Device storage: a caller region.
class BatchEngine {
 public:
  static size_t bytes_for(const std::vector<bdrs_solver>& members);
  // the same from the members' workspace layouts (before they are created)
  static size_t bytes_for_layouts(const std::vector<const Layout*>& layouts);
  // (re)binds the members: uploads descriptors and work lists into `ws`
  // (at least bytes_for(members) bytes) and, with a graph, captures one block
  hipError_t bind(const std::vector<bdrs_solver>& members, char* ws, int block_iters, bool use_graph,
                  hipStream_t st);
  // captures one block of the bound members as a graph (no-op if captured)
  hipError_t capture();
  bool captured() const { return exec_ != nullptr; }
  hipError_t run_block();                               // enqueue one block (+ certificates)
  hipError_t read_records(std::vector<double>& rec);    // D2H of the members' records, synchronises
  const std::vector<bdrs_solver>& members() const { return members_; }
  ~BatchEngine();

 private:
  hipError_t enqueue(hipStream_t st);
  std::vector<bdrs_solver> members_;
  BatchLayout B_{};
  char* ws_ = nullptr;
  hipStream_t st_ = nullptr;
  int dim_ = 0, iters_ = 0;
  int nrs_ = 0, ncs_ = 0, nrf_ = 0, ncf_ = 0, nce_ = 0;
  hipGraphExec_t exec_ = nullptr;
};

}  // namespace bdrs_host

struct bdrs_solver_ {
  bdrs_params prm;
  bdrs_host::Layout L;
  bdrs::LaunchCtx ctx;
  long long k = 0;          // finished iterations, refreshed from Ctrl::k by sync_k (the
                            // device counter is the truth: captured graphs advance it)
  double U_best = INFINITY, L_best = -INFINITY;
  long long kU = -1, kL = -1;
  bool packed_rows = false; // rows.A holds log alpha-hat of iteration k-1
  // sweep timing (bdrs_profile)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;  // created on demand, reused after each read
  size_t ev_used = 0;
  double prof_entries = 0.0;
  long long prof_sweeps = 0;
  // bdrs_solve: one captured block of blk_len iterations with its certificate
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t blk_exec = nullptr;
  int blk_len = 0;
  // BDRS_F_KEEP_BEST_STATE: relative gap of the retained state and its iteration count
  double best_rel = INFINITY;
  long long best_k = -1;
};
