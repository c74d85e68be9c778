// N of one spin sector of a given configuration, computed from its
// definition N = [e^V - G0 (e^V - 1)]^{-1}  (Eq. Nmatrix): M is built from the
// tabulated G0 (linear interpolation, the same lookup as the chains use) and
// inverted by the blocked Gauss-Jordan elimination with tournament pivoting of
// k_invert.hip.  Stateless: everything the call needs lives in the caller's
// workspace for the duration of the call.
#include <string.h>

#include <mutex>

#include "../../include/ctaux.h"
#include "ctaux_device.h"

namespace ctaux {

int model_error(const ctaux_model &m, int c, ctaux_batch *eb);
int create_error(int code, const char *fmt, ...);

// M[i][j] = delta_ij e^{V_i} - G0_{x_i x_j}(tau_i - tau_j) (e^{V_j} - 1) (Eq. Nmatrix),
// row-major with leading dimension n, from the caller's vertices as given.
__global__ __launch_bounds__(256) void k_build_M(const ChainDesc *dp, const ctaux_vertex *vx, int sec, int n,
                                                 double *W) {
  const ChainDesc &d = *dp;
  const int64_t total = static_cast<int64_t>(n) * n;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += gridDim.x * 256ll) {
    const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<int64_t>(i) * n);
    const ctaux_vertex vi = vx[i], vj = vx[j];
    const double evj = d.evd[sec][vj.s + 2];
    double v = -g0_interp(d, sec, vi.site, vj.site, vi.tau - vj.tau) * (evj - 1.0);
    if (i == j) v += d.evd[sec][vi.s + 2];
    W[e] = v;
  }
}

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace of one call: descriptor, the sector's tables, the site map, the
// configuration, the elimination item, M (n x n) and the elimination scratch.
struct BuildLayout {
  size_t desc, table, site_disp, verts, item, W, scratch, total;
};

BuildLayout build_layout(const ctaux_model &m, int n) {
  BuildLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.desc = take(sizeof(ChainDesc));
  L.table = take(sizeof(double) * static_cast<size_t>(m.n_disp) * m.n_tau);
  L.site_disp = take(sizeof(int32_t) * static_cast<size_t>(m.n_sites) * m.n_sites);
  L.verts = take(sizeof(ctaux_vertex) * n);
  L.item = take(sizeof(InvItem));
  L.W = take(sizeof(double) * static_cast<size_t>(n) * n);
  L.scratch = take(sizeof(double) * inv_scratch_doubles(n));
  L.total = off;
  return L;
}

}  // namespace

int build_args_error(const ctaux_model *model, const ctaux_vertex *config, int32_t n, int32_t sector) {
  if (!model) return create_error(CTAUX_EINVAL, "model is null");
  int rc = model_error(*model, 0, nullptr);
  if (rc) return rc;
  if (n < 0 || n > kBuildMaxOrder || sector < 0 || sector > 1 || (n > 0 && !config))
    return create_error(CTAUX_EINVAL, "need 0 <= n <= %d, sector 0 or 1 and a configuration", kBuildMaxOrder);
  for (int i = 0; i < n; ++i) {
    const ctaux_vertex &v = config[i];
    if (!(v.tau >= 0.0 && v.tau < model->beta) || v.site < 0 || v.site >= model->n_sites || (v.s != 1 && v.s != -1))
      return create_error(CTAUX_EINVAL, "vertex %d: need 0 <= tau < beta, 0 <= site < n_sites, s = +-1", i);
  }
  return CTAUX_OK;
}

size_t build_workspace_bytes(const ctaux_model &m, int n) { return build_layout(m, n).total; }

// The computation itself on a workspace of build_workspace_bytes(model, n) bytes
// (device memory; every byte the kernels read is written first).  Allocates
// nothing: the host values go to the device straight from the caller's arrays
// and from this frame.
int build_N_on(const ctaux_model *model, const ctaux_vertex *config, int32_t n, int32_t sector, double *dev_out,
               int32_t ld_out, char *ws, hipStream_t s) {
  const ctaux_model &m = *model;
  const BuildLayout L = build_layout(m, n);
  ChainDesc d;
  memset(&d, 0, sizeof d);
  d.beta = m.beta;
  d.K = m.K;
  d.gamma = acosh(1.0 + m.beta * m.U * m.n_sites / (2.0 * m.K));
  d.inv_h = static_cast<double>(m.n_tau - 1) / m.beta;
  for (int sec = 0; sec < 2; ++sec) {
    const double sigma = sec == 0 ? 1.0 : -1.0;
    for (int k = -2; k <= 2; ++k) d.evd[sec][k + 2] = exp(d.gamma * sigma * k);
  }
  d.nc = m.n_sites;
  d.n_tau = m.n_tau;
  d.n_disp = m.n_disp;
  d.g0[0] = d.g0[1] = reinterpret_cast<const double *>(ws + L.table);
  d.site_disp = reinterpret_cast<const int32_t *>(ws + L.site_disp);
  InvItem it;
  memset(&it, 0, sizeof it);
  double *W = reinterpret_cast<double *>(ws + L.W);
  inv_item_carve(it, W, n, n, reinterpret_cast<double *>(ws + L.scratch));
  const double *tab = sector == 0 ? m.g0_up : m.g0_dn;
  const InvItem *d_item = reinterpret_cast<const InvItem *>(ws + L.item);
#define BCHECK(call)                                                                                    \
  do {                                                                                                  \
    hipError_t e_ = (call);                                                                             \
    if (e_ != hipSuccess) return create_error(CTAUX_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));   \
  } while (0)
  BCHECK(hipMemcpyAsync(ws + L.desc, &d, sizeof d, hipMemcpyHostToDevice, s));
  BCHECK(hipMemcpyAsync(ws + L.table, tab, sizeof(double) * static_cast<size_t>(m.n_disp) * m.n_tau,
                        hipMemcpyHostToDevice, s));
  BCHECK(hipMemcpyAsync(ws + L.site_disp, m.site_disp, sizeof(int32_t) * m.n_sites * m.n_sites,
                        hipMemcpyHostToDevice, s));
  BCHECK(hipMemcpyAsync(ws + L.verts, config, sizeof(ctaux_vertex) * n, hipMemcpyHostToDevice, s));
  BCHECK(hipMemcpyAsync(ws + L.item, &it, sizeof it, hipMemcpyHostToDevice, s));
  BCHECK(hipStreamSynchronize(s));   // d and it live in this frame
  int dev = 0, n_cu = 0;
  BCHECK(hipGetDevice(&dev));
  BCHECK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t nn = static_cast<int64_t>(n) * n;
  const int g = static_cast<int>((nn + 255) / 256 < 2048 ? (nn + 255) / 256 : 2048);
  hipLaunchKernelGGL(k_build_M, dim3(g), dim3(256), 0, s, reinterpret_cast<const ChainDesc *>(ws + L.desc),
                     reinterpret_cast<const ctaux_vertex *>(ws + L.verts), sector, n, W);
  launch_invert(s, d_item, 1, n, n_cu);
  launch_inv_gather(s, d_item, dev_out, ld_out, n);
  BCHECK(hipGetLastError());
  int32_t flag = 0;
  BCHECK(hipMemcpyAsync(&flag, it.flag, sizeof flag, hipMemcpyDeviceToHost, s));
  BCHECK(hipStreamSynchronize(s));
#undef BCHECK
  if (flag) return create_error(CTAUX_ENUMERIC, "N^{-1} of the configuration is singular or not finite");
  return CTAUX_OK;
}

// ---- the allocation-free variant ----
// Device scratch of ctaux_build_N_noalloc: a file-scope array that every device
// the library runs on holds until the process ends.  Its host-side name is only
// a stand-in; kernels get the device address that hipGetSymbolAddress returns.
constexpr size_t kNoallocBytes = size_t{24} << 20;
constexpr int kNoallocMaxOrder = 1024;
static __device__ __align__(256) char scratch[kNoallocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device
// with that device current.
int scratch_ptr(char **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return create_error(CTAUX_EDEVICE, "no HIP device");
  if (dev < 0 || dev >= kMaxDevices) return create_error(CTAUX_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return create_error(CTAUX_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char *>(p);
  }
  *out = g_scratch_ptr[dev];
  return CTAUX_OK;
}

}  // namespace

}  // namespace ctaux

using namespace ctaux;

extern "C" {

size_t ctaux_build_N_workspace_bytes(const ctaux_model *model, int32_t n) {
  if (!model || model_error(*model, 0, nullptr) != CTAUX_OK || n < 0 || n > kBuildMaxOrder) return 0;
  return build_workspace_bytes(*model, n);
}

int ctaux_build_N(const ctaux_model *model, const ctaux_vertex *config, int32_t n, int32_t sector, double *dev_out,
                  int32_t ld_out, void *dev_workspace, size_t ws_bytes, void *hip_stream) {
  int rc = build_args_error(model, config, n, sector);
  if (rc) return rc;
  if (n == 0) return CTAUX_OK;
  if (!dev_out || ld_out < n) return create_error(CTAUX_EINVAL, "need an output and ld_out >= n");
  const size_t need = build_workspace_bytes(*model, n);
  if (!dev_workspace || ws_bytes < need)
    return create_error(CTAUX_ENOMEM, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (reinterpret_cast<uintptr_t>(dev_workspace) % 256 != 0)
    return create_error(CTAUX_EINVAL, "workspace must be 256-byte aligned");
  return build_N_on(model, config, n, sector, dev_out, ld_out, static_cast<char *>(dev_workspace),
                    static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"

extern "C" int ctaux_build_N_noalloc(const ctaux_model *model, const ctaux_vertex *config, int32_t n,
                                     int32_t sector, double *dev_out, int32_t ld_out, void *hip_stream) {
  int rc = build_args_error(model, config, n, sector);
  if (rc) return rc;
  if (n == 0) return CTAUX_OK;
  if (!dev_out || ld_out < n) return create_error(CTAUX_EINVAL, "need an output and ld_out >= n");
  if (n > kNoallocMaxOrder)
    return create_error(CTAUX_EINVAL, "n = %d exceeds %d, the largest order of the allocation-free variant", n,
                        kNoallocMaxOrder);
  const size_t need = build_workspace_bytes(*model, n);
  if (need > kNoallocBytes)
    return create_error(CTAUX_EINVAL, "this model and order need %zu bytes of scratch; the allocation-free "
                        "variant has %zu (tables too large)", need, kNoallocBytes);
  char *ws = nullptr;
  rc = scratch_ptr(&ws);
  if (rc) return rc;
  return build_N_on(model, config, n, sector, dev_out, ld_out, ws, static_cast<hipStream_t>(hip_stream));
}
