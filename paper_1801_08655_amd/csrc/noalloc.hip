// Allocation-free variant of the local solve entry point (helm_layer_solve_dev):
// the same substitution kernels, with every buffer they need beyond the
// caller's input and output taken from one file-scope device array instead of
// the handle's hipMalloc'ed workspace.
//
// The array holds, from its start, each at a 256-byte boundary:
//   - the layer table the kernels index (one LayerDev per layer; only the
//     solved layer's entry is written),
//   - X (the solve vector, n_loc x k), Z (the forward results, n_loc x k),
//   - the two depth-parity update buffers (ub_rows[0] x k, ub_rows[1] x k),
//   - the split-K partial products (scratch_rows x k),
// in the precision of the factors.  Every byte that the kernels read is
// written earlier in the same call (X by the copy-in, Z and the update
// buffers by the forward pass, the partials by the GEMM chunks), so nothing
// has to start at zero and the previous call's contents never matter.
#include <mutex>

#include "api_common.h"
#include "kernels.h"

namespace helm {

namespace {

// One copy per GPU, held until the process ends.  In host code `scratch`
// names a host-side stand-in: its device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[HELM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

__global__ void k_put_layer(LayerDev* dst, LayerDev v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst = v;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// Device address of the current device's copy of the array, looked up on the
// first call for that device (the factorization calls it with the handle's
// device current, so the solve entry point finds it cached).
void* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  HELM_REQUIRE(device >= 0 && device < kMaxDevices, HELM_EINVAL,
               "device ordinal out of range for the static scratch table");
  if (!g_scratch[device]) {
    int cur = -1;
    HELM_HIP(hipGetDevice(&cur));
    HELM_REQUIRE(cur == device, HELM_EINVAL, "static scratch looked up on another device");
    void* p = nullptr;
    HELM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    HELM_REQUIRE(p != nullptr, HELM_EHIP, "no device address for the static scratch");
    g_scratch[device] = p;
  }
  return g_scratch[device];
}

namespace {

template <typename T>
void solve_noalloc(Handle& H, int l, int k, const double2* r, double2* w, unsigned char* base) {
  const LayerPlan& P = H.G.layers[l];
  const LayerSet& S = *H.single_sets[l];
  const size_t e = H.elem, kk = (size_t)k;
  const size_t table = round256((size_t)H.G.L * sizeof(LayerDev));
  const size_t x_b = round256((size_t)P.n_loc * kk * e);
  const size_t u0_b = round256((size_t)std::max<long long>(P.ub_rows[0], 1) * kk * e);
  const size_t u1_b = round256((size_t)std::max<long long>(P.ub_rows[1], 1) * kk * e);
  const size_t sk_b = round256((size_t)std::max<long long>(S.scratch_rows, 1) * kk * e);
  const size_t need = table + 2 * x_b + u0_b + u1_b + sk_b;
  HELM_REQUIRE(need <= (size_t)HELM_NOALLOC_SCRATCH_BYTES, HELM_ENOMEM,
               "local solve needs " + std::to_string(need) +
                   " bytes of workspace, more than the static scratch of " +
                   std::to_string((size_t)HELM_NOALLOC_SCRATCH_BYTES) +
                   " bytes (use fewer columns or helm_layer_solve_dev)");
  LayerDev* tab = reinterpret_cast<LayerDev*>(base);
  LayerDev v = H.layers_h[l];
  unsigned char* p = base + table;
  v.X = p;
  p += x_b;
  v.Wt = p;
  p += x_b;
  v.Ub[0] = p;
  p += u0_b;
  v.Ub[1] = p;
  p += u1_b;
  void* splitk = p;
  hipLaunchKernelGGL(k_put_layer, dim3(1), dim3(64), 0, H.st, tab + l, v);
  kern::launch_local_to_X<T>(v, r, k, H.st);
  H.run_layers_t<T>(S, k, tab, splitk, nullptr, false);
  kern::launch_X_to_local<T>(v, w, k, H.st);
}

}  // namespace

}  // namespace helm

using namespace helm;

extern "C" int helm_layer_solve_noalloc_dev(helm_handle* h, int l, int k, const double* r_dev,
                                            double* w_dev) {
  return guard([&] {
    HELM_REQUIRE(h && r_dev && w_dev && k >= 1, HELM_EINVAL, "bad argument");
    Handle& H = h->impl;
    HELM_REQUIRE(l >= 0 && l < H.G.L, HELM_EINVAL, "layer index out of range");
    HELM_REQUIRE((int)H.single_sets.size() == H.G.L && H.single_sets[l], HELM_EINVAL,
                 "handle has no factorized layer plans");
    HELM_HIP(hipSetDevice(H.device));
    unsigned char* base = static_cast<unsigned char*>(noalloc_scratch(H.device));
    const double2* r = reinterpret_cast<const double2*>(r_dev);
    double2* w = reinterpret_cast<double2*>(w_dev);
    if (H.prec == HELM_FP64) solve_noalloc<double>(H, l, k, r, w, base);
    else solve_noalloc<float>(H, l, k, r, w, base);
    HELM_HIP(hipGetLastError());
    HELM_HIP(hipStreamSynchronize(H.st));
    return HELM_OK;
  });
}
