// amh_api.hip -- the C ABI of libamh.so (declared in include/amh.h): host-side
// validation, device buffers of a sampler context and stream-ordered launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "amh.h"
#include "amh_kernels.h"

namespace {

thread_local std::string g_last_error;

amh_status fail(amh_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
amh_status fail(amh_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(AMH_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

constexpr size_t kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950
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
  // trace
  int n_trace = 0;
  int trace_chain[4] = {-1, -1, -1, -1};
  double* tr_dE = nullptr;
  double* tr_delta = nullptr;
  uint8_t* tr_acc = nullptr;
  int64_t trace_cap = 0, trace_t0 = 0;
  double* tr_anchor = nullptr;
  int64_t trace_anchor_cap = 0, trace_anchor0 = 0;
};

namespace {

amh_status validate(const amh_config* c, int* G, int* W, size_t* lds) {
  if (!c) return fail(AMH_E_INVAL, "config is NULL");
  if (c->L < 2 || c->L > 1024) return fail(AMH_E_INVAL, "L=%d outside [2, 1024]", c->L);
  if (c->n_chains < 1) return fail(AMH_E_INVAL, "n_chains=%d < 1", c->n_chains);
  if (c->n_bins < 4 || c->n_bins > 64) return fail(AMH_E_INVAL, "n_bins=%d outside [4, 64]", c->n_bins);
  if (c->window_d < 0) return fail(AMH_E_INVAL, "window_d=%d < 0", c->window_d);
  if (!std::isfinite(c->d_min)) return fail(AMH_E_INVAL, "d_min not finite");
  if (!(c->bin_w > 0.0) || !std::isfinite(c->bin_w)) return fail(AMH_E_INVAL, "bin_w must be > 0");
  if (c->global_every < 0) return fail(AMH_E_INVAL, "global_every=%d < 0", c->global_every);
  if (c->anchor_every < 1) return fail(AMH_E_INVAL, "anchor_every=%d < 1", c->anchor_every);
  if (!(c->sigma >= 0.0) || !std::isfinite(c->sigma)) return fail(AMH_E_INVAL, "sigma must be finite and >= 0");
  if (!(c->T0 > 0.0) || !(c->T1 > 0.0) || !std::isfinite(c->T0) || !std::isfinite(c->T1))
    return fail(AMH_E_INVAL, "T0 and T1 must be finite and > 0");
  if (c->total_sweeps < 1 || c->total_sweeps > 0xFFFFFFFFLL)
    return fail(AMH_E_INVAL, "total_sweeps=%lld outside [1, 2^32-1]", (long long)c->total_sweeps);
  if ((uint64_t)c->chain_offset + (uint64_t)c->n_chains > 0x100000000ULL)
    return fail(AMH_E_INVAL, "chain_offset + n_chains exceeds 2^32");
  int g = c->chains_per_group;
  if (g != 0 && g != 1 && g != 2 && g != 4)
    return fail(AMH_E_INVAL, "chains_per_group=%d not in {0,1,2,4}", g);
  int w = c->waves_per_group;
  if (w < 0 || w > 8) return fail(AMH_E_INVAL, "waves_per_group=%d outside [0, 8]", w);
  if (g == 0) {
    g = 4;
    while (g > 1 && ((size_t)c->n_chains < (size_t)g * 256 ||
                     amh::sweep_lds_bytes(g, c->L, w ? w : (2 * g > 4 ? 2 * g : 4)) > kMaxLds))
      g >>= 1;
  }
  if (w == 0) w = 2 * g > 4 ? 2 * g : 4;
  if (w < g) return fail(AMH_E_INVAL, "waves_per_group=%d < chains_per_group=%d", w, g);
  const size_t need = amh::sweep_lds_bytes(g, c->L, w);
  if (need > kMaxLds)
    return fail(AMH_E_INVAL, "L=%d with %d chains per workgroup needs %zu bytes of LDS (> %zu)",
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
  delete x;
}

template <typename T>
amh_status dev_alloc(T** p, size_t count) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (count ? count : 1));
  if (e != hipSuccess) return fail(AMH_E_NOMEM, "hipMalloc(%zu bytes): %s", sizeof(T) * count, hipGetErrorString(e));
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

amh_status read_err(amh_ctx* x, unsigned int* out) {
  HIP_OK(hipStreamSynchronize(x->stream));
  HIP_OK(hipMemcpy(out, x->err, sizeof(unsigned int), hipMemcpyDeviceToHost));
  return AMH_OK;
}

}  // namespace

extern "C" {

const char* amh_last_error(void) { return g_last_error.c_str(); }

amh_status amh_init(const amh_config* cfg, const float* y_dev, const double* s0_dev, void* stream,
                    amh_ctx** out) {
  if (!out) return fail(AMH_E_INVAL, "out is NULL");
  *out = nullptr;
  int G = 0, W = 0;
  size_t lds = 0;
  amh_status st = validate(cfg, &G, &W, &lds);
  if (st != AMH_OK) return st;
  if (!y_dev) return fail(AMH_E_INVAL, "distogram table is NULL");
  amh_ctx* x = new amh_ctx;
  x->cfg = *cfg;
  x->stream = reinterpret_cast<hipStream_t>(stream);
  x->G = G;
  x->W = W;
  x->lds = lds;
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
  if (e == hipSuccess && s0_dev)
    e = hipMemcpyAsync(x->s, s0_dev, sizeof(double) * C * n, hipMemcpyDeviceToDevice, x->stream);
  if (e != hipSuccess) {
    free_ctx(x);
    return fail(AMH_E_DEVICE, "amh_init: %s", hipGetErrorString(e));
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
    return fail(AMH_E_NUMERIC, (err & amh::kErrTable) ? "distogram table holds a non-finite entry"
                                                       : "initial energy is not finite");
  }
  *out = x;
  return AMH_OK;
}

amh_status amh_sweep(amh_ctx* x, int64_t n_sweeps) {
  if (!x) return fail(AMH_E_INVAL, "ctx is NULL");
  if (n_sweeps < 0) return fail(AMH_E_INVAL, "n_sweeps < 0");
  if (x->t + n_sweeps > x->cfg.total_sweeps)
    return fail(AMH_E_INVAL, "sweep %lld + %lld passes total_sweeps=%lld", (long long)x->t,
                (long long)n_sweeps, (long long)x->cfg.total_sweeps);
  if (n_sweeps == 0) return AMH_OK;
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
  P.L = c.L;
  P.C = c.n_chains;
  P.half_window = c.window_d / 2;
  P.global_every = c.global_every;
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
  const dim3 grid((c.n_chains + x->G - 1) / x->G), block(64 * x->W);
  switch (x->G) {
    case 1:
      HIP_OK(hipFuncSetAttribute((const void*)amh::sweep_kernel<1>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)x->lds));
      hipLaunchKernelGGL(amh::sweep_kernel<1>, grid, block, x->lds, x->stream, P);
      break;
    case 2:
      HIP_OK(hipFuncSetAttribute((const void*)amh::sweep_kernel<2>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)x->lds));
      hipLaunchKernelGGL(amh::sweep_kernel<2>, grid, block, x->lds, x->stream, P);
      break;
    default:
      HIP_OK(hipFuncSetAttribute((const void*)amh::sweep_kernel<4>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)x->lds));
      hipLaunchKernelGGL(amh::sweep_kernel<4>, grid, block, x->lds, x->stream, P);
      break;
  }
  HIP_OK(hipGetLastError());
  x->t += n_sweeps;
  return AMH_OK;
}

amh_status amh_energy(amh_ctx* x, const double* s_in_dev, int32_t B, int32_t which,
                      double* V_out_dev, double* s_out_dev, float* cb_out_dev) {
  if (!x) return fail(AMH_E_INVAL, "ctx is NULL");
  if (B < 0) return fail(AMH_E_INVAL, "B < 0");
  amh::ConfParams P = conf_base(x);
  if (s_in_dev) {
    P.s_in = s_in_dev;
  } else {
    if (B != x->cfg.n_chains) return fail(AMH_E_INVAL, "B=%d must equal n_chains=%d", B, x->cfg.n_chains);
    if (which != 0 && which != 1) return fail(AMH_E_INVAL, "which=%d not in {0, 1}", which);
    P.s_in = which == 0 ? x->s : x->s_best;
  }
  P.V_out = V_out_dev;
  P.s_out = s_out_dev;
  P.cb_out = cb_out_dev;
  return launch_conf(P, B, x->stream);
}

amh_status amh_conformation(const double* s_dev, int32_t B, int32_t L, float* atoms_out_dev,
                            void* stream) {
  if (!s_dev || !atoms_out_dev) return fail(AMH_E_INVAL, "NULL pointer");
  if (B < 0 || L < 2 || L > 1024) return fail(AMH_E_INVAL, "B=%d, L=%d out of range", B, L);
  amh::ConfParams P{};
  P.L = L;
  P.s_in = s_dev;
  P.atoms_out = atoms_out_dev;
  return launch_conf(P, B, reinterpret_cast<hipStream_t>(stream));
}

amh_status amh_get_state(amh_ctx* x, double* s_dev, double* s_best_dev, double* v_dev,
                         int64_t* counters_dev, double* atoms_dev, int64_t* t_out) {
  if (!x) return fail(AMH_E_INVAL, "ctx is NULL");
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
  if (!x) return fail(AMH_E_INVAL, "ctx is NULL");
  if (t < 0 || t > x->cfg.total_sweeps) return fail(AMH_E_INVAL, "t=%lld out of range", (long long)t);
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

amh_status amh_set_target(amh_ctx* x, double target) {
  if (!x) return fail(AMH_E_INVAL, "ctx is NULL");
  if (std::isnan(target)) return fail(AMH_E_INVAL, "target is NaN");
  x->target = target;
  return AMH_OK;
}

amh_status amh_set_trace(amh_ctx* x, int32_t n, const int32_t* chain_ids, double* dE_dev,
                         double* delta_dev, uint8_t* acc_dev, int64_t capacity, double* anchor_dev,
                         int64_t anchor_capacity) {
  if (!x) return fail(AMH_E_INVAL, "ctx is NULL");
  if (n < 0 || n > 4) return fail(AMH_E_INVAL, "n=%d outside [0, 4]", n);
  if (n > 0 && (!chain_ids || !dE_dev || !delta_dev || !acc_dev || capacity < 0 || anchor_capacity < 0 ||
                (anchor_capacity > 0 && !anchor_dev)))
    return fail(AMH_E_INVAL, "trace buffers missing");
  for (int m = 0; m < 4; ++m) {
    x->trace_chain[m] = (m < n) ? chain_ids[m] : -1;
    if (m < n && (chain_ids[m] < -1 || chain_ids[m] >= x->cfg.n_chains))
      return fail(AMH_E_INVAL, "trace chain %d out of range", chain_ids[m]);
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

amh_status amh_poll(amh_ctx* x) {
  if (!x) return fail(AMH_E_INVAL, "ctx is NULL");
  unsigned int err = 0;
  amh_status st = read_err(x, &err);
  if (st != AMH_OK) return st;
  if (err & amh::kErrStall) return fail(AMH_E_DEVICE, "a pipelined localized sweep exceeded its wait bound");
  if (err) return fail(AMH_E_NUMERIC, "non-finite %s", (err & amh::kErrTable) ? "table entry" : "energy");
  return AMH_OK;
}

amh_status amh_info(amh_ctx* x, int32_t* G, int32_t* W, int32_t* lds, int64_t* t) {
  if (!x) return fail(AMH_E_INVAL, "ctx is NULL");
  if (G) *G = x->G;
  if (W) *W = x->W;
  if (lds) *lds = (int32_t)x->lds;
  if (t) *t = x->t;
  return AMH_OK;
}

amh_status amh_philox(const uint32_t* ctr_dev, int64_t n, uint64_t key, uint32_t* out_dev,
                      void* stream) {
  if (n < 0 || (n > 0 && (!ctr_dev || !out_dev))) return fail(AMH_E_INVAL, "bad philox arguments");
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
  (void)x; (void)s_dev; (void)B; (void)V_out_dev; (void)g_out_dev;
  return fail(AMH_E_UNSUPPORTED, "amh_grad is not provided by this build");
}

amh_status amh_submit(void* server, const void* job, uint64_t* job_id) {
  (void)server; (void)job; (void)job_id;
  return fail(AMH_E_UNSUPPORTED, "amh_submit is not provided by this build");
}

amh_status amh_destroy(amh_ctx* x) {
  if (!x) return AMH_OK;
  (void)hipStreamSynchronize(x->stream);
  free_ctx(x);
  return AMH_OK;
}

}  // extern "C"
