// amh_api.hip -- the C ABI of libamh.so (declared in include/amh.h): host-side
// validation, device buffers of a sampler context and stream-ordered launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "amh.h"
#include "amh_error.h"
#include "amh_grad.h"
#include "amh_kernels.h"

static_assert(sizeof(amh_config) == 120, "amh_config layout");
static_assert(sizeof(amh_lbfgs_opts) == 48, "amh_lbfgs_opts layout");

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace amh {
amh_status sfail(amh_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}
}  // namespace amh

namespace {

using amh::sfail;

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return sfail(AMH_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

constexpr size_t kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950
constexpr int kLocalWaves = 12;          // wavefronts of a localized-only sweep launch
constexpr int kConfThreads = 256;

int row_stride(int nb) { return ((nb + 2) + 3) & ~3; }   // nb values + 2 ghosts, 16-byte rows

}  // namespace

struct amh_ctx {
  amh_config cfg{};
  hipStream_t stream = nullptr;
  float* table = nullptr;
  float* ydev = nullptr;
  int stride = 0;
  double* s = nullptr;
  double* s_best = nullptr;
  double* atoms = nullptr;   // [C][L][4][3]
  double* v = nullptr;
  int64_t* counters = nullptr;
  unsigned int* err = nullptr;
  int64_t t = 0;
  double target = -INFINITY;
  int G = 1, W = 4;
  size_t lds = 0;
  // sum of every table row's no-contact value (far_sum_kernel)
  double vfar = 0.0;
  // launch shape of the localized-sweep kernel (wavefronts, LDS bytes)
  int W_local = 4;
  size_t lds_local = 0;
  // launch shape of the global-sweep kernel (chains and wavefronts per workgroup, LDS)
  int G_global = 1, W_global = 4;
  size_t lds_global = 0;
  // trace
  int n_trace = 0;
  int trace_chain[4] = {-1, -1, -1, -1};
  double* tr_dE = nullptr;
  double* tr_delta = nullptr;
  uint8_t* tr_acc = nullptr;
  int64_t trace_cap = 0, trace_t0 = 0;
  double* tr_anchor = nullptr;
  int64_t trace_anchor_cap = 0, trace_anchor0 = 0;
  int spin_limit = 1 << 24;   // bound of the pipelined sweeps' waits (amh_set_wait_bound)
  // L-BFGS workspace, grown on demand
  double* work = nullptr;
  size_t work_n = 0;
  // this device's copy of the library's fixed scratch array (amh_minimize_noalloc)
  double* scratch = nullptr;
  // caller's executed-work counters of the global sweeps (amh_set_work_counters)
  unsigned long long* work_counters = nullptr;
};

// Fixed scratch of amh_minimize_noalloc: the L-BFGS workspace of callers that cannot
// allocate.  Each device holds its own copy for the life of the process; host code
// reaches it only through the address hipGetSymbolAddress returns for the current
// device (the array's name in host code is not a device address).
static __device__ __align__(256) double scratch[amh::kNoallocScratchDoubles];

namespace {

std::mutex g_scratch_mu;
double* g_scratch_ptr[amh::kMaxDevices] = {};

// Device address of `scratch` on device `dev` (which must be current), looked up
// once per device and kept.
amh_status scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= amh::kMaxDevices) return sfail(AMH_E_DEVICE, "device %d outside [0, %d)", dev, amh::kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return sfail(AMH_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return AMH_OK;
}

}  // namespace

namespace {

// n_cu: compute units of the device (for the automatic launch shape).
amh_status validate(const amh_config* c, int n_cu, int* G, int* W, size_t* lds) {
  if (!c) return sfail(AMH_E_INVAL, "config is NULL");
  if (c->L < 2 || c->L > 1024) return sfail(AMH_E_INVAL, "L=%d outside [2, 1024]", c->L);
  if (c->n_chains < 1) return sfail(AMH_E_INVAL, "n_chains=%d < 1", c->n_chains);
  if (c->n_bins < 4 || c->n_bins > 64) return sfail(AMH_E_INVAL, "n_bins=%d outside [4, 64]", c->n_bins);
  if (c->window_d < 0) return sfail(AMH_E_INVAL, "window_d=%d < 0", c->window_d);
  if (!std::isfinite(c->d_min)) return sfail(AMH_E_INVAL, "d_min not finite");
  if (!(c->bin_w > 0.0) || !std::isfinite(c->bin_w)) return sfail(AMH_E_INVAL, "bin_w must be > 0");
  if (c->global_every < 0) return sfail(AMH_E_INVAL, "global_every=%d < 0", c->global_every);
  if (c->n_global < 0 || (c->global_every > 0 && c->n_global > c->global_every))
    return sfail(AMH_E_INVAL, "n_global=%d outside [0, global_every]", c->n_global);
  if (c->anchor_every < 1) return sfail(AMH_E_INVAL, "anchor_every=%d < 1", c->anchor_every);
  if (!(c->sigma >= 0.0) || !std::isfinite(c->sigma)) return sfail(AMH_E_INVAL, "sigma must be finite and >= 0");
  if (!(c->sigma_end >= 0.0) || !std::isfinite(c->sigma_end))
    return sfail(AMH_E_INVAL, "sigma_end must be finite and >= 0");
  if (c->n_cascade < 0 || c->n_cascade > 3) return sfail(AMH_E_INVAL, "n_cascade=%d outside [0, 3]", c->n_cascade);
  for (int i = 0; i < c->n_cascade; ++i)
    if (c->cascade_d[i] < 0) return sfail(AMH_E_INVAL, "cascade_d[%d]=%d < 0", i, c->cascade_d[i]);
  if (!(c->T0 > 0.0) || !(c->T1 > 0.0) || !std::isfinite(c->T0) || !std::isfinite(c->T1))
    return sfail(AMH_E_INVAL, "T0 and T1 must be finite and > 0");
  if (c->total_sweeps < 1 || c->total_sweeps > 0xFFFFFFFFLL)
    return sfail(AMH_E_INVAL, "total_sweeps=%lld outside [1, 2^32-1]", (long long)c->total_sweeps);
  if ((uint64_t)c->chain_offset + (uint64_t)c->n_chains > 0x100000000ULL)
    return sfail(AMH_E_INVAL, "chain_offset + n_chains exceeds 2^32");
  int g = c->chains_per_group;
  if (g != 0 && g != 1 && g != 2 && g != 4)
    return sfail(AMH_E_INVAL, "chains_per_group=%d not in {0,1,2,4}", g);
  int w = c->waves_per_group;
  if (w < 0 || w > 8) return sfail(AMH_E_INVAL, "waves_per_group=%d outside [0, 8]", w);
  if (g == 0) {
    g = 4;
    while (g > 1 && ((size_t)c->n_chains < (size_t)g * 256 ||
                     amh::sweep_lds_bytes(g, c->L, w ? w : (2 * g > 4 ? 2 * g : 4)) > kMaxLds))
      g >>= 1;
  }
  if (w == 0) {
    // eight waves (two per SIMD, the most the register budget allows) when the grid
    // gives each workgroup a compute unit of its own, else 2G (at least 4) so that
    // two workgroups share a compute unit
    const int64_t grid = ((int64_t)c->n_chains + g - 1) / g;
    w = 2 * g > 4 ? 2 * g : 4;
    if (grid <= n_cu && amh::sweep_lds_bytes(g, c->L, 8) <= kMaxLds) w = 8;
  }
  if (w < g) return sfail(AMH_E_INVAL, "waves_per_group=%d < chains_per_group=%d", w, g);
  const size_t need = amh::sweep_lds_bytes(g, c->L, w);
  if (need > kMaxLds)
    return sfail(AMH_E_INVAL, "L=%d with %d chains per workgroup needs %zu bytes of LDS (> %zu)",
                c->L, g, need, kMaxLds);
  *G = g;
  *W = w;
  *lds = need;
  return AMH_OK;
}

void free_ctx(amh_ctx* x) {
  if (!x) return;
  (void)hipFree(x->table); (void)hipFree(x->ydev); (void)hipFree(x->s); (void)hipFree(x->s_best); (void)hipFree(x->atoms);
  (void)hipFree(x->v); (void)hipFree(x->counters); (void)hipFree(x->err);
  (void)hipFree(x->work);
  delete x;
}

template <typename T>
amh_status dev_alloc(T** p, size_t count) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (count ? count : 1));
  if (e != hipSuccess) return sfail(AMH_E_NOMEM, "hipMalloc(%zu bytes): %s", sizeof(T) * count, hipGetErrorString(e));
  return AMH_OK;
}

amh::ConfParams conf_base(const amh_ctx* x) {
  amh::ConfParams P{};
  P.L = x->cfg.L;
  P.table = x->table;
  P.stride = x->stride;
  P.nb = x->cfg.n_bins;
  P.d_min = x->cfg.d_min;
  P.bin_w = x->cfg.bin_w;
  P.vfar = x->vfar;
  P.err = x->err;
  return P;
}

amh_status launch_conf(const amh::ConfParams& P, int B, hipStream_t st) {
  if (B <= 0) return AMH_OK;
  const size_t lds = amh::conf_lds_bytes(P.L, kConfThreads / 64);
  HIP_OK(hipFuncSetAttribute((const void*)amh::conf_energy_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(amh::conf_energy_kernel, dim3(B), dim3(kConfThreads), lds, st, P);
  HIP_OK(hipGetLastError());
  return AMH_OK;
}

amh::SweepParams sweep_params(const amh_ctx* x, int64_t n_sweeps) {
  const amh_config& c = x->cfg;
  amh::SweepParams P{};
  P.table = x->table;
  P.ydev = x->ydev;
  P.zrow = x->ydev + (size_t)c.L * (c.L - 1) / 2 * x->stride;
  P.stride = x->stride;
  P.nb = c.n_bins;
  P.inv_w = (float)(1.0 / c.bin_w);
  P.off = (float)((c.d_min + 0.5 * c.bin_w) / c.bin_w);
  P.tmax = (float)(c.n_bins - 1);
  {
    const double dfar = c.d_min + c.bin_w * (c.n_bins - 0.5);   // last knot
    P.d2far = (float)(dfar * dfar);
  }
  P.d_min = c.d_min;
  P.bin_w = c.bin_w;
  P.vfar = x->vfar;
  P.L = c.L;
  P.C = c.n_chains;
  P.half_window = c.window_d / 2;
  P.n_cascade = c.n_cascade;
  for (int i = 0; i < 3; ++i) P.cascade_hw[i] = i < c.n_cascade ? c.cascade_d[i] / 2 : 0;
  P.sigma_end = c.sigma_end;
  P.global_every = c.global_every;
  P.n_global = c.n_global < 1 ? 1 : c.n_global;
  P.anchor_every = c.anchor_every;
  P.sigma = c.sigma;
  P.T0 = c.T0;
  P.T1 = c.T1;
  P.S = c.total_sweeps;
  P.t0 = x->t;
  P.n_sweeps = n_sweeps;
  P.key0 = (uint32_t)c.seed;
  P.key1 = (uint32_t)(c.seed >> 32);
  P.chain_offset = c.chain_offset;
  P.spin_limit = x->spin_limit;
  P.target = x->target;
  P.s = x->s;
  P.s_best = x->s_best;
  P.atoms = x->atoms;
  P.v = x->v;
  P.counters = x->counters;
  P.err = x->err;
  P.n_trace = x->n_trace;
  for (int m = 0; m < 4; ++m) P.trace_chain[m] = x->trace_chain[m];
  P.tr_dE = x->tr_dE;
  P.tr_delta = x->tr_delta;
  P.tr_acc = x->tr_acc;
  P.trace_cap = x->trace_cap;
  P.trace_t0 = x->trace_t0;
  P.tr_anchor = x->tr_anchor;
  P.trace_anchor_cap = x->trace_anchor_cap;
  P.trace_anchor0 = x->trace_anchor0;
  P.work = x->work_counters;
  return P;
}

amh_status read_err(amh_ctx* x, unsigned int* out) {
  HIP_OK(hipStreamSynchronize(x->stream));
  HIP_OK(hipMemcpy(out, x->err, sizeof(unsigned int), hipMemcpyDeviceToHost));
  return AMH_OK;
}

}  // namespace

namespace {

// amh_minimize (workspace owned by the context, grown with hipMalloc) and
// amh_minimize_noalloc (workspace = this device's fixed scratch array).
amh_status minimize_impl(amh_ctx* x, double* s_dev, int32_t B, const amh_lbfgs_opts* o,
                         double* V_out_dev, int32_t* iters_out_dev, int32_t* status_out_dev,
                         double* f_trace_dev, double* x_trace_dev, bool no_alloc) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  if (!o) return sfail(AMH_E_INVAL, "opts is NULL");
  if (B < 0) return sfail(AMH_E_INVAL, "B < 0");
  if (!s_dev && B != x->cfg.n_chains)
    return sfail(AMH_E_INVAL, "B=%d must equal n_chains=%d when s is NULL", B, x->cfg.n_chains);
  if (o->n_iter < 0) return sfail(AMH_E_INVAL, "n_iter=%d < 0", o->n_iter);
  if (o->m < 1 || o->m > amh::kLbfgsMaxHistory)
    return sfail(AMH_E_INVAL, "m=%d outside [1, %d]", o->m, amh::kLbfgsMaxHistory);
  if (o->nonmonotone < 1 || o->nonmonotone > amh::kLbfgsMaxNonmonotone)
    return sfail(AMH_E_INVAL, "nonmonotone=%d outside [1, %d]", o->nonmonotone, amh::kLbfgsMaxNonmonotone);
  if (o->max_ls < 1) return sfail(AMH_E_INVAL, "max_ls=%d < 1", o->max_ls);
  if (!(o->c1 > 0.0 && o->c1 < 1.0)) return sfail(AMH_E_INVAL, "c1 must lie in (0, 1)");
  if (!(o->shrink > 0.0 && o->shrink < 1.0)) return sfail(AMH_E_INVAL, "shrink must lie in (0, 1)");
  if (!(o->gtol >= 0.0) || !std::isfinite(o->gtol)) return sfail(AMH_E_INVAL, "gtol must be finite and >= 0");
  if (!(o->step0 > 0.0) || !std::isfinite(o->step0)) return sfail(AMH_E_INVAL, "step0 must be finite and > 0");
  if (B == 0) return AMH_OK;
  const int L = x->cfg.L;
  const size_t need = amh::lbfgs_work_doubles(L, o->m) * (size_t)B;
  double* work = x->work;
  if (no_alloc) {
    if (need > (size_t)amh::kNoallocScratchDoubles)
      return sfail(AMH_E_INVAL,
                   "B=%d conformations of L=%d with m=%d need %zu workspace doubles; the fixed "
                   "scratch holds %lld (B (5 + 2m) 2L <= %lld)", B, L, o->m, need,
                   (long long)amh::kNoallocScratchDoubles, (long long)amh::kNoallocScratchDoubles);
    if (!x->scratch) return sfail(AMH_E_DEVICE, "the scratch array has no device address");
    work = x->scratch;
  } else if (need > x->work_n) {
    HIP_OK(hipStreamSynchronize(x->stream));
    (void)hipFree(x->work);
    x->work = nullptr;
    x->work_n = 0;
    amh_status st = dev_alloc(&x->work, need);
    if (st != AMH_OK) return st;
    x->work_n = need;
    work = x->work;
  }
  amh::LbfgsParams P{};
  P.L = L;
  P.s = s_dev ? s_dev : x->s;
  P.table = x->table;
  P.stride = x->stride;
  P.nb = x->cfg.n_bins;
  P.d_min = x->cfg.d_min;
  P.bin_w = x->cfg.bin_w;
  P.n_iter = o->n_iter;
  P.m = o->m;
  P.nonmonotone = o->nonmonotone;
  P.max_ls = o->max_ls;
  P.c1 = o->c1;
  P.shrink = o->shrink;
  P.gtol = o->gtol;
  P.step0 = o->step0;
  P.work = work;
  P.V = V_out_dev;
  P.iters = iters_out_dev;
  P.status = status_out_dev;
  P.f_trace = f_trace_dev;
  P.x_trace = x_trace_dev;
  P.err = x->err;
  if (!s_dev) {   // the context's chains: keep V, the best state and the coordinates current
    P.v_state = x->v;
    P.s_best = x->s_best;
  }
  const size_t lds = amh::lbfgs_lds_bytes(L, amh::kGradThreads / 64, o->m, o->nonmonotone);
  if (lds > kMaxLds) return sfail(AMH_E_INVAL, "L=%d needs %zu bytes of LDS for L-BFGS", L, lds);
  HIP_OK(hipFuncSetAttribute((const void*)amh::lbfgs_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  hipLaunchKernelGGL(amh::lbfgs_kernel, dim3(B), dim3(amh::kGradThreads), lds, x->stream, P);
  HIP_OK(hipGetLastError());
  if (!s_dev) {
    amh::ConfParams cp{};
    cp.L = L;
    cp.s_in = x->s;
    cp.atoms64_out = x->atoms;
    return launch_conf(cp, B, x->stream);
  }
  return AMH_OK;
}

}  // namespace

extern "C" {

const char* amh_last_error(void) { return g_last_error.c_str(); }

amh_status amh_init(const amh_config* cfg, const float* y_dev, const double* s0_dev, void* stream,
                    amh_ctx** out) {
  if (!out) return sfail(AMH_E_INVAL, "out is NULL");
  *out = nullptr;
  int G = 0, W = 0;
  size_t lds = 0;
  int dev = 0, n_cu = 0;
  const bool have_dev = hipGetDevice(&dev) == hipSuccess;
  if (!have_dev || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      n_cu < 1)
    n_cu = 256;
  amh_status st = validate(cfg, n_cu, &G, &W, &lds);
  if (st != AMH_OK) return st;
  if (!y_dev) return sfail(AMH_E_INVAL, "distogram table is NULL");
  if (!have_dev) return sfail(AMH_E_DEVICE, "no current HIP device");
  double* scratch_dev = nullptr;
  if ((st = scratch_address(dev, &scratch_dev)) != AMH_OK) return st;
  amh_ctx* x = new amh_ctx;
  x->cfg = *cfg;
  x->scratch = scratch_dev;
  x->stream = reinterpret_cast<hipStream_t>(stream);
  x->G = G;
  x->W = W;
  x->lds = lds;
  // localized sweeps run with kLocalWaves wavefronts (consecutive sweeps of a block
  // pipelined over more stages) where their LDS fits
  x->W_local = amh::sweep_lds_bytes_local(G, cfg->L, kLocalWaves) <= kMaxLds ? kLocalWaves : W;
  x->lds_local = amh::sweep_lds_bytes_local(G, cfg->L, x->W_local);
  // global sweeps of an automatically shaped context: two workgroups of two chains
  // and four wavefronts per CU where their LDS fits, so that one workgroup runs
  // while the other waits at a barrier
  x->G_global = G;
  x->W_global = W;
  x->lds_global = lds;
  if (cfg->chains_per_group == 0 && cfg->waves_per_group == 0 && G == 4 && W == 8 &&
      2 * amh::sweep_lds_bytes(2, cfg->L, 4) <= kMaxLds) {
    x->G_global = 2;
    x->W_global = 4;
    x->lds_global = amh::sweep_lds_bytes(2, cfg->L, 4);
  }
  const int L = cfg->L, C = cfg->n_chains, n = 2 * L;
  const int64_t P = (int64_t)L * (L - 1) / 2;
  x->stride = row_stride(cfg->n_bins);
  if ((st = dev_alloc(&x->table, (size_t)P * x->stride)) != AMH_OK ||
      (st = dev_alloc(&x->ydev, (size_t)(P + 1) * x->stride)) != AMH_OK ||
      (st = dev_alloc(&x->s, (size_t)C * n)) != AMH_OK ||
      (st = dev_alloc(&x->s_best, (size_t)C * n)) != AMH_OK ||
      (st = dev_alloc(&x->atoms, (size_t)C * L * 12)) != AMH_OK ||
      (st = dev_alloc(&x->v, (size_t)C * 2)) != AMH_OK ||
      (st = dev_alloc(&x->counters, (size_t)C * 4)) != AMH_OK ||
      (st = dev_alloc(&x->err, 1)) != AMH_OK) {
    free_ctx(x);
    return st;
  }
  hipError_t e = hipMemsetAsync(x->err, 0, sizeof(unsigned int), x->stream);
  if (e == hipSuccess)   // row P of the deviation table is the zero row
    e = hipMemsetAsync(x->ydev + (size_t)P * x->stride, 0, sizeof(float) * x->stride, x->stream);
  if (e == hipSuccess) {
    const int64_t work = P * x->stride;
    int blocks = (int)((work + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(amh::ingest_kernel, dim3(blocks), dim3(256), 0, x->stream, y_dev, P,
                       cfg->n_bins, x->stride, x->table, x->ydev, x->err);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {   // the energy of the all-far conformation, read back once
    double* d_vfar = nullptr;
    e = hipMalloc(reinterpret_cast<void**>(&d_vfar), sizeof(double));
    if (e == hipSuccess) {
      hipLaunchKernelGGL(amh::far_sum_kernel, dim3(1), dim3(512), 0, x->stream, x->table, P, x->stride,
                         cfg->n_bins, d_vfar);
      e = hipGetLastError();
      if (e == hipSuccess)
        e = hipMemcpyAsync(&x->vfar, d_vfar, sizeof(double), hipMemcpyDeviceToHost, x->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
      (void)hipFree(d_vfar);
    }
  }
  if (e == hipSuccess && s0_dev)
    e = hipMemcpyAsync(x->s, s0_dev, sizeof(double) * C * n, hipMemcpyDeviceToDevice, x->stream);
  if (e != hipSuccess) {
    free_ctx(x);
    return sfail(AMH_E_DEVICE, "amh_init: %s", hipGetErrorString(e));
  }
  amh::ConfParams cp = conf_base(x);
  cp.s_in = s0_dev ? x->s : nullptr;
  cp.s_out = s0_dev ? nullptr : x->s;
  cp.atoms64_out = x->atoms;
  cp.v_state = x->v;
  cp.counters = x->counters;
  cp.s_best = x->s_best;
  if ((st = launch_conf(cp, C, x->stream)) != AMH_OK) { free_ctx(x); return st; }
  unsigned int err = 0;
  if ((st = read_err(x, &err)) != AMH_OK) { free_ctx(x); return st; }
  if (err) {
    free_ctx(x);
    return sfail(AMH_E_NUMERIC, (err & amh::kErrTable) ? "distogram table holds a non-finite entry"
                                                       : "initial energy is not finite");
  }
  *out = x;
  return AMH_OK;
}

amh_status amh_sweep(amh_ctx* x, int64_t n_sweeps) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  if (n_sweeps < 0) return sfail(AMH_E_INVAL, "n_sweeps < 0");
  if (x->t + n_sweeps > x->cfg.total_sweeps)
    return sfail(AMH_E_INVAL, "sweep %lld + %lld passes total_sweeps=%lld", (long long)x->t,
                (long long)n_sweeps, (long long)x->cfg.total_sweeps);
  if (n_sweeps == 0) return AMH_OK;
  const amh::SweepParams P0 = sweep_params(x, n_sweeps);
  const amh_config& c = x->cfg;
  const dim3 grid((c.n_chains + x->G - 1) / x->G), block(64 * x->W);
  const int wl = x->W_local;
  const size_t lds_l = x->lds_local;
  // one launch per run of sweeps of one kind (localized or global), in order on the
  // stream; a launch boundary between two sweeps does not change any result
  for (int64_t t = P0.t0; t < P0.t0 + P0.n_sweeps;) {
    const bool glob = amh::is_global(P0, t);
    int64_t e = t + 1;
    while (e < P0.t0 + P0.n_sweeps && amh::is_global(P0, e) == glob) ++e;
    amh::SweepParams P = P0;
    P.t0 = t;
    P.n_sweeps = e - t;
    const void* fn = nullptr;
    switch (glob ? x->G_global : x->G) {
      case 1: fn = glob ? (const void*)amh::sweep_kernel<1, amh::kSweepGlobal>
                        : (const void*)amh::sweep_kernel<1, amh::kSweepLocal>; break;
      case 2: fn = glob ? (const void*)amh::sweep_kernel<2, amh::kSweepGlobal>
                        : (const void*)amh::sweep_kernel<2, amh::kSweepLocal>; break;
      default: fn = glob ? (const void*)amh::sweep_kernel<4, amh::kSweepGlobal>
                         : (const void*)amh::sweep_kernel<4, amh::kSweepLocal>; break;
    }
    const size_t lds = glob ? x->lds_global : lds_l;
    const dim3 gg((c.n_chains + x->G_global - 1) / x->G_global);
    HIP_OK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    void* args[] = {&P};
    HIP_OK(hipLaunchKernel(fn, glob ? gg : grid, dim3(64 * (glob ? x->W_global : wl)), args, lds, x->stream));
    t = e;
  }
  HIP_OK(hipGetLastError());
  x->t += n_sweeps;
  return AMH_OK;
}

amh_status amh_energy(amh_ctx* x, const double* s_in_dev, int32_t B, int32_t which,
                      double* V_out_dev, double* s_out_dev, float* cb_out_dev) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  if (B < 0) return sfail(AMH_E_INVAL, "B < 0");
  amh::ConfParams P = conf_base(x);
  if (s_in_dev) {
    P.s_in = s_in_dev;
  } else {
    if (B != x->cfg.n_chains) return sfail(AMH_E_INVAL, "B=%d must equal n_chains=%d", B, x->cfg.n_chains);
    if (which != 0 && which != 1) return sfail(AMH_E_INVAL, "which=%d not in {0, 1}", which);
    P.s_in = which == 0 ? x->s : x->s_best;
  }
  P.V_out = V_out_dev;
  P.s_out = s_out_dev;
  P.cb_out = cb_out_dev;
  return launch_conf(P, B, x->stream);
}

amh_status amh_conformation(const double* s_dev, int32_t B, int32_t L, float* atoms_out_dev,
                            void* stream) {
  if (!s_dev || !atoms_out_dev) return sfail(AMH_E_INVAL, "NULL pointer");
  if (B < 0 || L < 2 || L > 1024) return sfail(AMH_E_INVAL, "B=%d, L=%d out of range", B, L);
  amh::ConfParams P{};
  P.L = L;
  P.s_in = s_dev;
  P.atoms_out = atoms_out_dev;
  return launch_conf(P, B, reinterpret_cast<hipStream_t>(stream));
}

amh_status amh_get_state(amh_ctx* x, double* s_dev, double* s_best_dev, double* v_dev,
                         int64_t* counters_dev, double* atoms_dev, int64_t* t_out) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  const size_t C = x->cfg.n_chains, n = 2 * (size_t)x->cfg.L;
  const auto D2D = hipMemcpyDeviceToDevice;
  if (s_dev) HIP_OK(hipMemcpyAsync(s_dev, x->s, sizeof(double) * C * n, D2D, x->stream));
  if (s_best_dev) HIP_OK(hipMemcpyAsync(s_best_dev, x->s_best, sizeof(double) * C * n, D2D, x->stream));
  if (v_dev) HIP_OK(hipMemcpyAsync(v_dev, x->v, sizeof(double) * C * 2, D2D, x->stream));
  if (counters_dev) HIP_OK(hipMemcpyAsync(counters_dev, x->counters, sizeof(int64_t) * C * 4, D2D, x->stream));
  if (atoms_dev) HIP_OK(hipMemcpyAsync(atoms_dev, x->atoms, sizeof(double) * C * x->cfg.L * 12, D2D, x->stream));
  if (t_out) *t_out = x->t;
  return AMH_OK;
}

amh_status amh_set_state(amh_ctx* x, const double* s_dev, const double* s_best_dev,
                         const double* v_dev, const int64_t* counters_dev, const double* atoms_dev,
                         int64_t t) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  if (t < 0 || t > x->cfg.total_sweeps) return sfail(AMH_E_INVAL, "t=%lld out of range", (long long)t);
  const size_t C = x->cfg.n_chains, n = 2 * (size_t)x->cfg.L;
  const auto D2D = hipMemcpyDeviceToDevice;
  if (s_dev) HIP_OK(hipMemcpyAsync(x->s, s_dev, sizeof(double) * C * n, D2D, x->stream));
  if (s_best_dev) HIP_OK(hipMemcpyAsync(x->s_best, s_best_dev, sizeof(double) * C * n, D2D, x->stream));
  if (v_dev) HIP_OK(hipMemcpyAsync(x->v, v_dev, sizeof(double) * C * 2, D2D, x->stream));
  if (counters_dev) HIP_OK(hipMemcpyAsync(x->counters, counters_dev, sizeof(int64_t) * C * 4, D2D, x->stream));
  if (atoms_dev) {
    HIP_OK(hipMemcpyAsync(x->atoms, atoms_dev, sizeof(double) * C * x->cfg.L * 12, D2D, x->stream));
  } else if (s_dev) {
    amh::ConfParams P{};
    P.L = x->cfg.L;
    P.s_in = x->s;
    P.atoms64_out = x->atoms;
    amh_status st = launch_conf(P, (int)C, x->stream);
    if (st != AMH_OK) return st;
  }
  x->t = t;
  return AMH_OK;
}

amh_status amh_perturb(amh_ctx* x, double amplitude, uint32_t tag) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  if (!(amplitude >= 0.0) || !std::isfinite(amplitude)) return sfail(AMH_E_INVAL, "amplitude must be finite and >= 0");
  const amh_config& c = x->cfg;
  const int64_t total = (int64_t)c.n_chains * 2 * c.L;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(amh::perturb_kernel, dim3(blocks), dim3(256), 0, x->stream, x->s, total, 2 * c.L,
                     c.chain_offset, tag, (uint32_t)c.seed, (uint32_t)(c.seed >> 32), amplitude);
  HIP_OK(hipGetLastError());
  amh::ConfParams P = conf_base(x);   // rebuild coordinates, re-anchor V, keep the best
  P.s_in = x->s;
  P.atoms64_out = x->atoms;
  P.v_state = x->v;
  P.s_best = x->s_best;
  P.keep_best = 1;
  return launch_conf(P, c.n_chains, x->stream);
}

amh_status amh_set_wait_bound(amh_ctx* x, int32_t polls) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  if (polls < 1 || polls > (1 << 24)) return sfail(AMH_E_INVAL, "polls=%d outside [1, 2^24]", polls);
  x->spin_limit = polls;
  return AMH_OK;
}

amh_status amh_set_target(amh_ctx* x, double target) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  if (std::isnan(target)) return sfail(AMH_E_INVAL, "target is NaN");
  x->target = target;
  return AMH_OK;
}

amh_status amh_set_trace(amh_ctx* x, int32_t n, const int32_t* chain_ids, double* dE_dev,
                         double* delta_dev, uint8_t* acc_dev, int64_t capacity, double* anchor_dev,
                         int64_t anchor_capacity) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  if (n < 0 || n > 4) return sfail(AMH_E_INVAL, "n=%d outside [0, 4]", n);
  if (n > 0 && (!chain_ids || !dE_dev || !delta_dev || !acc_dev || capacity < 0 || anchor_capacity < 0 ||
                (anchor_capacity > 0 && !anchor_dev)))
    return sfail(AMH_E_INVAL, "trace buffers missing");
  for (int m = 0; m < 4; ++m) {
    x->trace_chain[m] = (m < n) ? chain_ids[m] : -1;
    if (m < n && (chain_ids[m] < -1 || chain_ids[m] >= x->cfg.n_chains))
      return sfail(AMH_E_INVAL, "trace chain %d out of range", chain_ids[m]);
  }
  x->n_trace = n;
  x->tr_dE = dE_dev;
  x->tr_delta = delta_dev;
  x->tr_acc = acc_dev;
  x->trace_cap = capacity;
  x->trace_t0 = x->t;
  x->tr_anchor = anchor_dev;
  x->trace_anchor_cap = anchor_capacity;
  x->trace_anchor0 = x->t / x->cfg.anchor_every + 1;
  return AMH_OK;
}

amh_status amh_set_work_counters(amh_ctx* x, int64_t* counters_dev) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  x->work_counters = reinterpret_cast<unsigned long long*>(counters_dev);
  return AMH_OK;
}

amh_status amh_poll(amh_ctx* x) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  unsigned int err = 0;
  amh_status st = read_err(x, &err);
  if (st != AMH_OK) return st;
  if (err & amh::kErrStall) return sfail(AMH_E_DEVICE, "a pipelined localized sweep exceeded its wait bound");
  if (err) return sfail(AMH_E_NUMERIC, "non-finite %s", (err & amh::kErrTable) ? "table entry" : "energy");
  return AMH_OK;
}

amh_status amh_info(amh_ctx* x, int32_t* G, int32_t* W, int32_t* lds, int64_t* t) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  if (G) *G = x->G;
  if (W) *W = x->W;
  if (lds) *lds = (int32_t)x->lds;
  if (t) *t = x->t;
  return AMH_OK;
}

amh_status amh_info_launches(amh_ctx* x, int32_t* local_G, int32_t* local_W, int32_t* local_lds,
                             int32_t* global_G, int32_t* global_W, int32_t* global_lds) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  if (local_G) *local_G = x->G;
  if (local_W) *local_W = x->W_local;
  if (local_lds) *local_lds = (int32_t)x->lds_local;
  if (global_G) *global_G = x->G_global;
  if (global_W) *global_W = x->W_global;
  if (global_lds) *global_lds = (int32_t)x->lds_global;
  return AMH_OK;
}

amh_status amh_philox(const uint32_t* ctr_dev, int64_t n, uint64_t key, uint32_t* out_dev,
                      void* stream) {
  if (n < 0 || (n > 0 && (!ctr_dev || !out_dev))) return sfail(AMH_E_INVAL, "bad philox arguments");
  if (n == 0) return AMH_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(amh::philox_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), ctr_dev, n, (uint32_t)key,
                     (uint32_t)(key >> 32), out_dev);
  HIP_OK(hipGetLastError());
  return AMH_OK;
}

amh_status amh_grad(amh_ctx* x, const double* s_dev, int32_t B, double* V_out_dev, double* g_out_dev) {
  if (!x) return sfail(AMH_E_INVAL, "ctx is NULL");
  if (B < 0) return sfail(AMH_E_INVAL, "B < 0");
  if (!s_dev && B != x->cfg.n_chains)
    return sfail(AMH_E_INVAL, "B=%d must equal n_chains=%d when s is NULL", B, x->cfg.n_chains);
  if (!V_out_dev && !g_out_dev) return sfail(AMH_E_INVAL, "V_out and g_out are both NULL");
  if (B == 0) return AMH_OK;
  amh::GradParams P{};
  P.L = x->cfg.L;
  P.s = s_dev ? s_dev : x->s;
  P.table = x->table;
  P.stride = x->stride;
  P.nb = x->cfg.n_bins;
  P.d_min = x->cfg.d_min;
  P.bin_w = x->cfg.bin_w;
  P.V = V_out_dev;
  P.g = g_out_dev;
  P.err = x->err;
  const size_t lds = amh::grad_lds_bytes(P.L, amh::kGradThreads / 64);
  if (lds > kMaxLds) return sfail(AMH_E_INVAL, "L=%d needs %zu bytes of LDS for the gradient", P.L, lds);
  HIP_OK(hipFuncSetAttribute((const void*)amh::grad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  hipLaunchKernelGGL(amh::grad_kernel, dim3(B), dim3(amh::kGradThreads), lds, x->stream, P);
  HIP_OK(hipGetLastError());
  return AMH_OK;
}

amh_status amh_minimize(amh_ctx* x, double* s_dev, int32_t B, const amh_lbfgs_opts* o,
                        double* V_out_dev, int32_t* iters_out_dev, int32_t* status_out_dev,
                        double* f_trace_dev, double* x_trace_dev) {
  return minimize_impl(x, s_dev, B, o, V_out_dev, iters_out_dev, status_out_dev, f_trace_dev,
                       x_trace_dev, false);
}

amh_status amh_minimize_noalloc(amh_ctx* x, double* s_dev, int32_t B, const amh_lbfgs_opts* o,
                                double* V_out_dev, int32_t* iters_out_dev, int32_t* status_out_dev,
                                double* f_trace_dev, double* x_trace_dev) {
  return minimize_impl(x, s_dev, B, o, V_out_dev, iters_out_dev, status_out_dev, f_trace_dev,
                       x_trace_dev, true);
}

amh_status amh_destroy(amh_ctx* x) {
  if (!x) return AMH_OK;
  (void)hipStreamSynchronize(x->stream);
  free_ctx(x);
  return AMH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: several contexts (proteins of different lengths) advanced by one launch
// per launch shape.

namespace {

constexpr int kRing = 8;   // pinned descriptor staging buffers in flight
constexpr int kMaxRuns = 8;   // runs of one kind of sweep per call with split launches
// launch plans: 0 = each context's own shape, then uniform (chains per group, waves)
constexpr int kPlans = 6;
constexpr int kPlanShape[kPlans][2] = {{0, 0}, {1, 4}, {2, 4}, {2, 8}, {4, 4}, {4, 8}};

}  // namespace

struct amh_batch {
  std::vector<amh_ctx*> m;
  hipStream_t stream = nullptr;
  int plan = 0;
  struct Launch {
    int G = 1, W = 4;
    size_t lds = 0;
    size_t lds_local = 0;   // LDS of a localized-only launch with kLocalWaves wavefronts
    int n_wg = 0;
    int2* d_map = nullptr;
  };
  std::vector<Launch> launches;
  amh::SweepParams* d_desc = nullptr;
  amh::SweepParams* h_desc[kRing] = {};
  hipEvent_t ev[kRing] = {};
  bool ev_used[kRing] = {};
  int ring = 0;
};

namespace {

void free_launches(amh_batch* b) {
  for (auto& l : b->launches) (void)hipFree(l.d_map);
  b->launches.clear();
}

void free_batch(amh_batch* b) {
  if (!b) return;
  free_launches(b);
  (void)hipFree(b->d_desc);
  for (int i = 0; i < kRing; ++i) {
    if (b->h_desc[i]) (void)hipHostFree(b->h_desc[i]);
    if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
  }
  delete b;
}

void member_shape(const amh_ctx* x, int plan, int* G, int* W) {
  if (plan == 0) { *G = x->G; *W = x->W; return; }
  int g = kPlanShape[plan][0], w = kPlanShape[plan][1];
  while (g > 1 && amh::sweep_lds_bytes(g, x->cfg.L, w) > kMaxLds) g >>= 1;
  *G = g;
  *W = w;
}

// Work of one chain group per sweep, in pair evaluations (orders the grid only).
double member_cost(const amh_ctx* x) {
  const double L = x->cfg.L, h = x->cfg.window_d / 2;
  const int ge = x->cfg.global_every;
  const double fg = ge > 0 ? (double)(x->cfg.n_global < 1 ? 1 : x->cfg.n_global) / ge : 0.0;
  const double global = L * L * L / 3.0 * fg;
  const double local = 2.0 * L * h * (h + 1) * (1.0 - fg);
  return global + local;
}

amh_status build_launches(amh_batch* b, int plan) {
  HIP_OK(hipStreamSynchronize(b->stream));
  free_launches(b);
  std::vector<std::pair<int, int>> shapes;
  std::vector<int> shape_of(b->m.size());
  for (size_t i = 0; i < b->m.size(); ++i) {
    int G, W;
    member_shape(b->m[i], plan, &G, &W);
    auto it = std::find(shapes.begin(), shapes.end(), std::make_pair(G, W));
    shape_of[i] = (int)(it - shapes.begin());
    if (it == shapes.end()) shapes.emplace_back(G, W);
  }
  for (size_t s = 0; s < shapes.size(); ++s) {
    amh_batch::Launch l;
    l.G = shapes[s].first;
    l.W = shapes[s].second;
    std::vector<std::pair<double, int2>> items;
    for (size_t i = 0; i < b->m.size(); ++i) {
      if (shape_of[i] != (int)s) continue;
      const amh_ctx* x = b->m[i];
      l.lds = std::max(l.lds, amh::sweep_lds_bytes(l.G, x->cfg.L, l.W));
      l.lds_local = std::max(l.lds_local, amh::sweep_lds_bytes_local(l.G, x->cfg.L, kLocalWaves));
      const int groups = (x->cfg.n_chains + l.G - 1) / l.G;
      for (int g = 0; g < groups; ++g) items.push_back({member_cost(x), make_int2((int)i, g)});
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const auto& a, const auto& c) { return a.first > c.first; });
    std::vector<int2> map;
    for (auto& it : items) map.push_back(it.second);
    l.n_wg = (int)map.size();
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&l.d_map), sizeof(int2) * map.size());
    if (e != hipSuccess) return sfail(AMH_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
    b->launches.push_back(l);
    HIP_OK(hipMemcpy(l.d_map, map.data(), sizeof(int2) * map.size(), hipMemcpyHostToDevice));
  }
  b->plan = plan;
  return AMH_OK;
}

template <int G, int MODE>
amh_status launch_batch(const amh_batch* b, const amh_batch::Launch& l, const amh::SweepParams* descs,
                        int W, size_t lds) {
  HIP_OK(hipFuncSetAttribute((const void*)amh::sweep_batch_kernel<G, MODE>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((amh::sweep_batch_kernel<G, MODE>), dim3(l.n_wg), dim3(64 * W), lds, b->stream, descs,
                     (const int2*)l.d_map);
  HIP_OK(hipGetLastError());
  return AMH_OK;
}

template <int MODE>
amh_status launch_batch_mode(const amh_batch* b, const amh_batch::Launch& l, const amh::SweepParams* descs,
                             int W, size_t lds) {
  return l.G == 1 ? launch_batch<1, MODE>(b, l, descs, W, lds)
         : l.G == 2 ? launch_batch<2, MODE>(b, l, descs, W, lds)
                    : launch_batch<4, MODE>(b, l, descs, W, lds);
}

}  // namespace

extern "C" {

amh_status amh_batch_create(amh_ctx* const* ctxs, int32_t n, amh_batch** out) {
  if (!out) return sfail(AMH_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!ctxs || n < 1) return sfail(AMH_E_INVAL, "need at least one context");
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return sfail(AMH_E_INVAL, "context %d is NULL", i);
    if (ctxs[i]->stream != ctxs[0]->stream)
      return sfail(AMH_E_INVAL, "context %d is on another stream than context 0", i);
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return sfail(AMH_E_INVAL, "context %d appears twice", i);
  }
  amh_batch* b = new amh_batch;
  b->m.assign(ctxs, ctxs + n);
  b->stream = ctxs[0]->stream;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&b->d_desc), sizeof(amh::SweepParams) * kMaxRuns * n);
  for (int i = 0; e == hipSuccess && i < kRing; ++i) {
    e = hipHostMalloc(reinterpret_cast<void**>(&b->h_desc[i]), sizeof(amh::SweepParams) * kMaxRuns * n);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    free_batch(b);
    return sfail(AMH_E_NOMEM, "amh_batch_create: %s", hipGetErrorString(e));
  }
  amh_status st = build_launches(b, 0);
  if (st != AMH_OK) { free_batch(b); return st; }
  *out = b;
  return AMH_OK;
}

amh_status amh_batch_sweep_each(amh_batch* b, const int64_t* n_sweeps) {
  if (!b) return sfail(AMH_E_INVAL, "batch is NULL");
  if (!n_sweeps) return sfail(AMH_E_INVAL, "n_sweeps is NULL");
  int64_t most = 0;
  for (size_t i = 0; i < b->m.size(); ++i) {
    const amh_ctx* x = b->m[i];
    if (n_sweeps[i] < 0) return sfail(AMH_E_INVAL, "member %zu: n_sweeps < 0", i);
    if (x->t + n_sweeps[i] > x->cfg.total_sweeps)
      return sfail(AMH_E_INVAL, "member %zu: sweep %lld + %lld passes total_sweeps=%lld", i,
                   (long long)x->t, (long long)n_sweeps[i], (long long)x->cfg.total_sweeps);
    most = std::max(most, n_sweeps[i]);
  }
  if (most == 0) return AMH_OK;
  const size_t nm = b->m.size();
  // Split launches (localized-only and global-only kernels, one launch per run of
  // one kind) when every member advances by the same count through the same pattern
  // of localized and global sweeps; else one launch of the kernel that runs any
  // sweeps.  The results are the same either way.  Descriptors go up kMaxRuns runs
  // at a time (stream order keeps an upload behind the launches that read the last).
  std::vector<std::pair<int64_t, bool>> runs;   // (length, global)
  bool split = true;
  for (size_t i = 1; i < nm && split; ++i) split = n_sweeps[i] == n_sweeps[0];
  if (split) {
    std::vector<amh::SweepParams> P0(nm);
    for (size_t i = 0; i < nm; ++i) P0[i] = sweep_params(b->m[i], n_sweeps[i]);
    for (int64_t o = 0; o < most && split; ++o) {
      const bool g = amh::is_global(P0[0], P0[0].t0 + o);
      for (size_t i = 1; i < nm && split; ++i) split = amh::is_global(P0[i], P0[i].t0 + o) == g;
      if (!split) break;
      if (!runs.empty() && runs.back().second == g) ++runs.back().first;
      else runs.emplace_back(1, g);
    }
  }
  for (const auto& l : b->launches) split = split && l.lds_local <= kMaxLds;
  if (!split) runs.assign(1, std::make_pair(most, false));
  int64_t off = 0;
  for (size_t r0 = 0; r0 < runs.size(); r0 += kMaxRuns) {
    const size_t nset = std::min(runs.size() - r0, (size_t)kMaxRuns);
    const int slot = b->ring;
    if (b->ev_used[slot]) HIP_OK(hipEventSynchronize(b->ev[slot]));
    for (size_t r = 0; r < nset; ++r) {
      for (size_t i = 0; i < nm; ++i) {
        amh::SweepParams P = sweep_params(b->m[i], n_sweeps[i]);
        if (split) {
          P.t0 += off;
          P.n_sweeps = runs[r0 + r].first;
        }
        b->h_desc[slot][r * nm + i] = P;
      }
      off += runs[r0 + r].first;
    }
    HIP_OK(hipMemcpyAsync(b->d_desc, b->h_desc[slot], sizeof(amh::SweepParams) * nset * nm,
                          hipMemcpyHostToDevice, b->stream));
    HIP_OK(hipEventRecord(b->ev[slot], b->stream));
    b->ev_used[slot] = true;
    b->ring = (slot + 1) % kRing;
    for (size_t r = 0; r < nset; ++r) {
      const amh::SweepParams* descs = b->d_desc + r * nm;
      for (const auto& l : b->launches) {
        amh_status st = !split ? launch_batch_mode<amh::kSweepMixed>(b, l, descs, l.W, l.lds)
                        : runs[r0 + r].second
                            ? launch_batch_mode<amh::kSweepGlobal>(b, l, descs, l.W, l.lds)
                            : launch_batch_mode<amh::kSweepLocal>(b, l, descs, kLocalWaves, l.lds_local);
        if (st != AMH_OK) return st;
      }
    }
  }
  for (size_t i = 0; i < nm; ++i) b->m[i]->t += n_sweeps[i];
  return AMH_OK;
}

amh_status amh_batch_sweep(amh_batch* b, int64_t n_sweeps) {
  if (!b) return sfail(AMH_E_INVAL, "batch is NULL");
  if (n_sweeps < 0) return sfail(AMH_E_INVAL, "n_sweeps < 0");
  std::vector<int64_t> n(b->m.size(), n_sweeps);
  return amh_batch_sweep_each(b, n.data());
}

amh_status amh_batch_tune(amh_batch* b, int64_t sweeps_per_trial, float* ms_out, int32_t* plan_out) {
  if (!b) return sfail(AMH_E_INVAL, "batch is NULL");
  if (sweeps_per_trial < 1) return sfail(AMH_E_INVAL, "sweeps_per_trial < 1");
  for (size_t i = 0; i < b->m.size(); ++i) {
    const amh_ctx* x = b->m[i];
    if (x->t + kPlans * sweeps_per_trial > x->cfg.total_sweeps)
      return sfail(AMH_E_INVAL, "member %zu has fewer than %lld sweeps left for tuning", i,
                  (long long)(kPlans * sweeps_per_trial));
  }
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  int best = 0;
  float best_ms = 0.0f;
  amh_status st = AMH_OK;
  for (int p = 0; p < kPlans && st == AMH_OK; ++p) {
    if ((st = build_launches(b, p)) != AMH_OK) break;
    if (hipEventRecord(e0, b->stream) != hipSuccess) { st = sfail(AMH_E_DEVICE, "hipEventRecord"); break; }
    if ((st = amh_batch_sweep(b, sweeps_per_trial)) != AMH_OK) break;
    float ms = 0.0f;
    if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = sfail(AMH_E_DEVICE, "timing a tuning trial failed");
      break;
    }
    if (ms_out) ms_out[p] = ms;
    if (p == 0 || ms < best_ms) { best = p; best_ms = ms; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != AMH_OK) return st;
  if ((st = build_launches(b, best)) != AMH_OK) return st;
  if (plan_out) *plan_out = best;
  return AMH_OK;
}

amh_status amh_batch_set_plan(amh_batch* b, int32_t plan) {
  if (!b) return sfail(AMH_E_INVAL, "batch is NULL");
  if (plan < 0 || plan >= kPlans) return sfail(AMH_E_INVAL, "plan=%d outside [0, %d)", plan, kPlans);
  return build_launches(b, plan);
}

amh_status amh_batch_info(const amh_batch* b, int32_t* plan, int32_t* n_launches, int32_t* workgroups) {
  if (!b) return sfail(AMH_E_INVAL, "batch is NULL");
  int wg = 0;
  for (const auto& l : b->launches) wg += l.n_wg;
  if (plan) *plan = b->plan;
  if (n_launches) *n_launches = (int)b->launches.size();
  if (workgroups) *workgroups = wg;
  return AMH_OK;
}

amh_status amh_batch_destroy(amh_batch* b) {
  if (!b) return AMH_OK;
  (void)hipStreamSynchronize(b->stream);
  free_batch(b);
  return AMH_OK;
}

}  // extern "C"
