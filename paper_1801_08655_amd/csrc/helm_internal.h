// Internal declarations of the polarized-traces library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/helm.h"

namespace helm {

using cd = std::complex<double>;

// ---------------------------------------------------------------------------
// error handling: no exception crosses the C ABI
// ---------------------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};
void set_last_error(const std::string& s);
const char* last_error_cstr();

#define HELM_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::helm::Error{HELM_EHIP, std::string(#call) + ": " +              \
                                         hipGetErrorString(e_)};              \
  } while (0)

#define HELM_REQUIRE(cond, code, text)                                        \
  do {                                                                        \
    if (!(cond)) throw ::helm::Error{(code), (text)};                         \
  } while (0)

// ---------------------------------------------------------------------------
// device-side descriptors (plain old data, copied to device memory)
// ---------------------------------------------------------------------------

// One front of a layer's nested-dissection tree.  Its frontal matrix has
// s fully summed variables (the separator) followed by b boundary
// variables (face neighbours of its subtree box, all in ancestors).
struct FrontDev {
  int s, b;          // pivots, boundary size
  int off;           // ND index of the first pivot inside its layer
  int layer;         // owning layer
  long long fac;     // element offset of [F11^-1; -F21 F11^-1] ((s+b) x s, col-major)
  long long ws;      // element offset of the frontal matrix in its workspace
  int ws_parity;     // which factorization workspace (depth parity)
  int bidx;          // offset of the b sorted ND indices of the boundary
  int inv[2];        // offsets of the front-row -> child-boundary maps (-1: none)
  int child[2];      // global ids of the children (-1: none)
  long long wt;      // row offset into the layer's gathered-pivot buffer
  long long ub;      // row offset into the layer's update buffer (depth parity)
  int ub_parity;     // depth parity
  int pad;
};

// The launch lists of a solve may carry flags in the top bits of a front id
// (solves pruned to the fronts that touch their sources and read-outs): the
// front's child 0 or 1 contributes nothing (its subtree holds no source), or
// its forward result Z(S) is zero (no source below it, but a read-out).
constexpr int kFrontIdMask = (1 << 27) - 1;
constexpr int kSkipChild0 = 1 << 27;
constexpr int kSkipChild1 = 1 << 28;
constexpr int kZeroZ = 1 << 29;

// Split of one front's substitution GEMMs along K (the pivot / boundary
// dimension) into chunks computed by separate workgroups; partial products
// go to a scratch area and are summed in a fixed order.
struct SolveTask {
  int nch_f, kc_f;   // forward: chunks, chunk length
  int nch_b, kc_b;   // backward
  long long scr_f;   // scratch row offset of the forward partials (nch_f x (s+b) rows)
  long long scr_b;   // scratch row offset of the backward partials (nch_b x s rows)
};

// Per-layer base pointers for kernels that touch several layers at once.
struct LayerDev {
  void* fac;          // factor store base (complex elements of the precision)
  void* X;            // solve vector, n_loc x k, ND order, column fastest
  void* Wt;           // gathered pivots (forward)
  void* Ub[2];        // update / boundary-gather buffers (depth parity)
  const int* bidx;    // boundary ND indices
  const int* inv;     // front-row -> child-boundary maps
  const int* nat2nd;  // natural local index -> ND index
  const int* nd2nat;  // ND index -> natural local index
  const double2* bz;  // beta_z at the extended layer's planes (t)
  const double2* bzh; // beta_z at half planes (t + 1), index p <-> p - 1/2
  int n_loc;
  int t;              // planes of the extended layer
  int lo;             // first global plane of the extended layer
  int s, e;           // bulk planes (global)
};

// Geometry shared by the volume kernels.
struct GridDev {
  int nx, ny, nz;
  double h, omega;
  const double* m;    // squared slowness (global grid)
  const double2* bx;  // beta_x at nodes (nx)
  const double2* bxh; // beta_x at half nodes (nx + 1), index i <-> i - 1/2
  const double2* by;
  const double2* byh;
  const double2* bz;  // global beta_z (nz), bzh (nz + 1)
  const double2* bzh;
};

// ---------------------------------------------------------------------------
// host-side plan
// ---------------------------------------------------------------------------
struct Box {
  int lo[3], hi[3];   // half-open, local coordinates (x, y, z)
  long long volume() const {
    return (long long)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
  }
};

struct FrontHost {
  Box box;        // subtree box
  Box sep;        // separator (pivots); equals box for leaves
  int s = 0, b = 0, off = 0, depth = 0;
  int parent = -1;
  int child[2] = {-1, -1};
};

struct LayerPlan {
  int index = 0;
  int s = 0, e = 0, lo = 0, hi = 0;  // global planes
  int t = 0;                         // extended planes
  int n_loc = 0;
  std::vector<FrontHost> fronts;     // post-order (children before parents)
  std::vector<int> nat2nd, nd2nat;
  std::vector<int> bidx;             // concatenated boundaries
  std::vector<int> bidx_off;         // per front
  std::vector<int> inv;              // concatenated front-row -> child maps
  std::vector<int> inv_off;          // per front and slot (2 per front)
  std::vector<long long> fac_off;    // per front
  long long fac_elems = 0;
  int max_depth = 0;
  std::vector<std::vector<int>> by_depth;  // local front ids, s descending
  long long wt_rows = 0;             // max over depths of sum s
  long long ub_rows[2] = {0, 0};     // max over same-parity depths of sum b
  std::vector<long long> wt_off, ub_off;  // per front
  long long max_front = 0;
  double factor_flops = 0;           // real flops of an LU of every front:
                                     // 4 (2/3 s^3 + 2 s^2 b + 2 s b^2)
  double gj_flops = 0;               // real flops the blocked Gauss-Jordan
                                     // sweep executes (skipped tiles excluded)
  double solve_elems = 0;            // factor elements read by one solve
};

// Pivot block of the factorization's Gauss-Jordan sweep (columns per step).
constexpr int kPivotBlock = 64;

// Real flops the sweep of one front (s pivots, b boundary variables)
// executes: per block step of nbf pivots, the rank-nbf update of every
// 64 x 64 tile it does not skip (tiles inside the pivot rows or columns, and
// tiles of eliminated rows x boundary columns, whose values are never read
// again), plus the two products with the inverted pivot block.
double gj_front_flops(int s, int b, int nb);

struct Geometry {
  int nx = 0, ny = 0, nz = 0;
  double h = 0, omega = 0, C = 0;
  int pml = 0, L = 0, alpha = 0;
  std::vector<cd> bx, bxh, by, byh, bz, bzh;   // global tables
  std::vector<std::vector<cd>> lbz, lbzh;       // per layer z tables
  std::vector<LayerPlan> layers;
};

// Builds layer bounds, beta tables and the nested-dissection plan of every
// layer.  Throws Error(HELM_EINVAL) for impossible geometries.
void build_geometry(Geometry& G, const helm_grid& g, double omega, int pml,
                    int n_layers, int alpha, double C, int leaf);

namespace kern {
template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };
}  // namespace kern

}  // namespace helm
