// The factorization handle: resident factors, plans and launch lists.
#pragma once

#include <map>
#include <memory>
#include <vector>

#include "helm_internal.h"
#include "kernels.h"

namespace helm {

// Device allocation owned by the handle.
struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem();
  void alloc(size_t b);
  void release();
  template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};

// A pair of timing events, destroyed with the scope that owns them.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair();
  EventPair(const EventPair&) = delete;
  EventPair& operator=(const EventPair&) = delete;
  ~EventPair();
  // milliseconds between recording a and b on the stream
  double elapsed_ms(hipStream_t st) const;
};

// Fronts of one depth over a set of layers, for the substitutions.
struct DepthList {
  int n = 0;
  DevMem ids;                 // global front ids (backward: all fronts)
  DevMem tasks;               // SolveTask per front (K splits, scratch offsets)
  DevMem pBw, rB;             // backward GEMM tiles incl. K chunks; reduce tiles
  int nS = 0;                 // forward: fronts with children (extend-add gather)
  DevMem idsS;
  int nL = 0;                 // forward: every front (GEMM)
  DevMem idsL, tasksL;
  DevMem pSB;                 // prefix of 64-row tiles of s+b of the gathered fronts
  DevMem pF, rF;              // forward GEMM tiles incl. K chunks; reduce tiles
  int tSB = 0, tF = 0, tBw = 0, tRF = 0, tRB = 0;
  int bwd_bm = 64;            // row tile of the backward GEMM at this depth
  double sum_s = 0, sum_b = 0, sum_sbs = 0, sum_bs = 0;  // work counts, all fronts
  double fs_s = 0, fs_b = 0, fs_sbs = 0;    // fronts with children
  double fl_s = 0, fl_b = 0, fl_sbs = 0;    // all fronts (forward GEMM)
  long long scratch_rows = 0;
};

// Kernel classes timed with HIP events when HELM_FLAG_PROFILE is set.
enum KClass {
  K_FWD_GATHER, K_FWD_GEMM, K_FWD_REDUCE, K_BWD_GEMM, K_BWD_REDUCE,
  K_SWEEP_GEMM, K_PANEL,
  K_SWAP_JO, K_UPDATE_OJ, K_EXTEND_ADD, K_ORIG, K_STORE, K_NCLASS
};
struct KStat {
  long long launches = 0;
  double ms = 0, flops = 0, bytes = 0;
};
struct PendingEvent {
  int cls;
  hipEvent_t a, b;
  double flops, bytes;
};
// Interface-plane masks of a pruned local solve.
constexpr int kPruneTop = 1, kPruneBottom = 2;
constexpr int kPruneAll = 4;   // sources anywhere in the layer (no forward pruning)

struct LayerSet {
  std::vector<int> layers;
  int max_depth = 0;
  double elems = 0;             // factor elements one solve reads
  long long scratch_rows = 0;   // max over depths
  std::vector<std::unique_ptr<DepthList>> depth;
};

// Fronts of one depth of a factorization group, sorted by s (descending),
// so that the fronts still active at block step k are a prefix of the list.
struct FactorDepth {
  int n = 0;
  std::vector<int> s_sorted;
  std::vector<int> pFull_h, pCol_h;
  DevMem ids, pFull, pCol, pRow, pStore, panel_off, perm_off;
  int tRow = 0, tStore = 0;
  long long panel_total = 0, perm_total = 0;
};

struct Handle {
  Geometry G;
  helm_options opt{};
  int prec = HELM_MIXED;          // HELM_FP64: complex128 fronts, else complex64
  size_t elem = 8;                // bytes of one complex element of the factors
  hipStream_t st = nullptr;
  bool own_stream = false;
  hipStream_t cap_st = nullptr;   // graph captures (non-blocking, see solve_layers)
  // Launch sequences are captured into graphs unless a server lane drives
  // the handle: a lane's capture on its own thread would make the caller's
  // device-wide synchronizations fail while it lasts (measured: the lanes
  // run at the same rate without graphs).
  bool capture = true;
  int device = 0;
  int nb = kPivotBlock;           // pivot block of the Gauss-Jordan sweep

  // geometry on device
  DevMem m, bx, bxh, by, byh, bz, bzh, Bcoef;
  std::vector<std::unique_ptr<DevMem>> lbz, lbzh, nat2nd, nd2nat, bidx, inv, fac;
  std::vector<int> front_base;   // global id of each layer's first front
  int n_fronts = 0;
  DevMem fronts;                 // FrontDev[n_fronts]
  std::vector<FrontDev> fronts_h;
  std::vector<LayerDev> layers_h;
  DevMem layers_d;
  GridDev grid{};

  // solve workspace (per layer) for up to kcap columns
  int kcap = 0;
  std::vector<std::unique_ptr<DevMem>> X, Wt, Ub0, Ub1;
  std::map<std::vector<int>, std::unique_ptr<LayerSet>> sets;
  DevMem scratch;                // split-K partial products
  // captured substitution sequences: (set, k) -> executable graph
  struct GraphKey {
    const LayerSet* set;
    int k;
    bool operator<(const GraphKey& o) const {
      return set < o.set || (set == o.set && k < o.k);
    }
  };
  std::map<GraphKey, hipGraphExec_t> graphs;
  void clear_graphs();
  // column-tile widths of the substitution GEMMs per depth, per (set, k);
  // width 1 is the vector path (k <= 4)
  struct TileChoice {
    int fwd_bn = 64, bwd_bn = 64;
    bool tuned = false;
    double t_fwd[4] = {0, 0, 0, 0}, t_bwd[4] = {0, 0, 0, 0};   // us per width 1/16/32/64
  };
  std::map<GraphKey, std::vector<TileChoice>> tiles;
  // measured choices shared by every depth list of the same front-size
  // bucket: (k, fronts, log2 mean s and mean b in quarter steps, bwd row tile)
  std::map<std::vector<long long>, TileChoice> tuned;
  const std::vector<TileChoice>& tile_plan(const LayerSet& set, int k);
  template <typename T> void autotune_t(const LayerSet& set, int k,
                                        std::vector<TileChoice>& plan);
  template <typename T> void launch_fwd(const DepthList& D, const FrontDev* fr,
                                        const LayerDev* ld, int k, void* scr, int bn,
                                        hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
  template <typename T> void launch_bwd(const DepthList& D, const FrontDev* fr,
                                        const LayerDev* ld, int k, void* scr, int bn,
                                        hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

  // kernel timing (HELM_FLAG_PROFILE: every class; HELM_FLAG_PROFILE_FWD:
  // the forward substitution GEMM only), one bit per KClass
  unsigned profile_mask = 0;
  void set_profile(int flags);
  // three-product complex64 GEMMs: substitutions (unless HELM_FLAG_GEMM_4M),
  // factorization sweep (unless HELM_FLAG_FACTOR_4M)
  bool gemm3m = false, factor3m = false;
  bool profile() const { return profile_mask != 0; }
  KStat kstats[K_NCLASS];
  std::vector<PendingEvent> pending;
  std::vector<hipEvent_t> ev_free;
  hipEvent_t take_event();     // from the pool, not recorded
  hipEvent_t record_event();
  bool timed(int cls) const { return (profile_mask >> cls) & 1u; }
  hipEvent_t prof_begin(int cls);
  void prof_end(int cls, hipEvent_t a, double flops, double bytes);
  void collect_profile();

  // statistics
  double factor_seconds = 0;
  // wall time of the other phases of helm_factorize (host plans, device
  // set-up, single-layer launch lists)
  double symbolic_seconds = 0, setup_seconds = 0, lists_seconds = 0;
  double factor_flops = 0;        // LU count of every front (algorithmic)
  double factor_gj_flops = 0;     // flops the Gauss-Jordan sweep executes
  // pivot statistics of the last factorization (device: status flag, then
  // the bit patterns of min and max |pivot|^2 and of max |diagonal entry|^2
  // of the assembled operator)
  double pivot_min = 0, pivot_max = 0, diag_max = 0;
  int zero_pivots = 0;
  long long layer_solves = 0;
  double solve_bytes = 0;
  size_t bytes_factors = 0;

  ~Handle();
  void init_device(const helm_options& o);
  void upload_geometry(const double* m_src, bool m_on_device);
  void build_fronts();
  void factorize();
  template <typename T> void factorize_t();
  void ensure_workspace(int k);
  const LayerSet& layer_set(const std::vector<int>& layers);
  // launch lists of a single-layer solve whose sources lie on the interface
  // planes of `src` and whose result is read on those of `read` (kPrune*)
  const LayerSet& pruned_set(int l, int src, int read);
  struct Prune {
    std::vector<char> fwd, bwd;   // per global front: in the forward / backward pass
  };
  std::unique_ptr<LayerSet> make_set(const std::vector<int>& layers, const Prune* pr);
  std::map<std::vector<int>, std::unique_ptr<LayerSet>> psets;
  // multi-RHS solve of the layers in `set` on their X buffers (k columns)
  void solve_layers(const LayerSet& set, int k);
  template <typename T> void solve_layers_t(const LayerSet& set, int k);
  template <typename T> void run_layers_t(const LayerSet& set, int k, const LayerDev* ld,
                                          void* scr, const TileChoice* tp, bool timing);
  // the single-layer sets, built with the factors (used without allocation
  // by the allocation-free local solve)
  std::vector<const LayerSet*> single_sets;
  // an existing layer set, or null (no allocation)
  const LayerSet* find_layer_set(const std::vector<int>& layers) const;
  void upload_layers();
  double solve_elems(const LayerSet& set) const;
};

size_t plan_factor_elems(const Geometry& G);
// frontal workspace per depth of one layer, and its bytes for a group
std::pair<std::vector<long long>, std::vector<long long>> layer_workspace(const LayerPlan& P,
                                                                          int nb);
size_t workspace_bytes(const std::vector<long long>& a, const std::vector<long long>& p,
                       size_t elem);
size_t plan_bytes_per_rhs(const Geometry& G, size_t elem);
size_t plan_pair_bytes_per_rhs(const Geometry& G);
// per-slot reservation of a server or batch lane: the solve workspace of one
// column plus the Krylov and sweep vectors of the lane's narrower widths
size_t lane_bytes_per_slot(const Geometry& G, size_t elem);

}  // namespace helm
