// C ABI of the retrieval library (declared in include/tm.h): argument
// validation, context and workspace, twiddle tables, and the host-side
// sequencing of the device kernels. All arithmetic of the method runs in
// the device kernels; the host only launches them in order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>


#include "../../include/tm.h"
#include "aux.hpp"
#include "foci.hpp"
#include "batch.hpp"
#include "grids.hpp"
#include "lbfgs.hpp"
#include "mlp.hpp"
#include "phase.hpp"
#include "pre.hpp"
#include "row_kernels.hpp"
#include "wnet.hpp"

constexpr int TM_PROF_MODES = 24;  // row-kernel modes 0..16, 20 L-BFGS direction, 21 L-BFGS step

struct tm_ctx {
  int device = 0;
  std::string err;
  tmk::cx<float>* tw32 = nullptr;
  tmk::cx<double>* tw64 = nullptr;
  struct Slot {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<int, Slot> ws;
  // per-launch event timing of the fused row kernels (tm_profile_enable)
  bool prof = false;
  struct Rec {
    int mode;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double acc_ms[TM_PROF_MODES] = {0};
  int64_t acc_n[TM_PROF_MODES] = {0};
  std::map<int, int> variant;  // (L1 << 8 | L2) -> launch configuration (bit 0: FFT digit-order variant)
  double* pinned = nullptr;    // 8 doubles of pinned host memory for read-backs
  int phase_band = 1;             // band evaluation of the defocus model when the pupil's box is small
  // The captured phase iteration of the last tm_phase_offset_correct call, reused
  // while everything it captured (pointers, sizes, options, band plan) is unchanged.
  struct PhaseGraph {
    std::vector<double> key;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
  } pg;
  int32_t ph_iters = 0, ph_evals = 0;  // accepted iterations and evaluations of the last phase solve
  int32_t ph_iters_req = -1;           // the iteration count that solve was asked for
  void* scratch = nullptr;             // device address of the no-allocation scratch on this device
  int32_t wtab_n = 0;                  // learned weight table (tm_set_weight_table): points, 0 = none
  float wtab_xmax = 0.f;               // and its range [0, xmax]
};

constexpr int PHASE_GRAPH_ITERS = 10;  // phase L-BFGS iterations captured per graph replay

// Scratch of tm_retrieve_noalloc: per-row monitoring sums [rows][NSUM] float,
// then the FP64 residual sums [rows][2] double. One copy per device, held
// until the process ends. Host code never passes `scratch` itself to a
// kernel (in host code it names a host-side stand-in): it uses the device
// address that tm_create looks up for the context's device.
constexpr size_t NA_SUMS_BYTES = (size_t)TM_NOALLOC_MAX_ROWS * tmk::NSUM * sizeof(float);
constexpr size_t NA_S64_OFF = (NA_SUMS_BYTES + 255) / 256 * 256;
constexpr size_t NA_SCRATCH_BYTES = NA_S64_OFF + (size_t)TM_NOALLOC_MAX_ROWS * 2 * sizeof(double);
static __device__ __align__(256) unsigned char scratch[NA_SCRATCH_BYTES];

namespace {
constexpr int NA_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NA_MAX_DEVICES] = {};  // device address of `scratch`, per device
}  // namespace

static void phase_graph_release(tm_ctx* c) {
  if (c->pg.exec) hipGraphExecDestroy(c->pg.exec);
  if (c->pg.g) hipGraphDestroy(c->pg.g);
  if (c->pg.cap) hipStreamDestroy(c->pg.cap);
  c->pg = tm_ctx::PhaseGraph{};
}

namespace {

constexpr int TW_MAX = 8192;  // longest FFT axis
thread_local std::string g_create_err;

int fail(tm_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  else g_create_err = buf;
  return code;
}

int hipfail(tm_ctx* c, int e, const char* what) {
  return fail(c, TM_EHIP, "%s: %s", what, hipGetErrorString((hipError_t)e));
}

#define HIPCHK(ctx, expr)                                 \
  do {                                                    \
    int _e = (int)(expr);                                 \
    if (_e != 0) return hipfail(ctx, _e, #expr);          \
  } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Workspace slot `id` of at least `bytes` bytes (grown on demand). Growing
// synchronises the device first so that no queued kernel still uses it.
void* ws_get(tm_ctx* c, int id, size_t bytes) {
  auto& s = c->ws[id];
  if (s.bytes >= bytes && s.p) return s.p;
  if (s.p) {
    hipDeviceSynchronize();
    hipFree(s.p);
    s.p = nullptr;
    s.bytes = 0;
  }
  size_t want = bytes < 256 ? 256 : bytes;
  if (hipMalloc(&s.p, want) != hipSuccess) {
    s.p = nullptr;
    return nullptr;
  }
  s.bytes = want;
  return s.p;
}

enum WsId {
  WS_SUMS = 1, WS_SUMS64, WS_ROWSUM, WS_ROWMEAN, WS_VPREV,
  WS_LB_G, WS_LB_GP, WS_LB_D, WS_LB_S, WS_LB_Y, WS_LB_SC, WS_LB_ST, WS_TPREV, WS_VSCALE, WS_LZ_V, WS_LZ_H, WS_LZ_Y, WS_PRE_PART,
  WS_PRE_COUNT, WS_FOCI_U, WS_FOCI_E, WS_DENSE_Y, WS_PROP_X, WS_PROP_H, WS_PROP_ONES, WS_WTAB,
  WS_PH_BASE = 100
};

int check_dims(tm_ctx* c, const tm_dims& d, tmk::row_launcher* fn) {
  if (d.n1 < 1 || d.n2 < 1 || !is_pow2(d.n1) || !is_pow2(d.n2))
    return fail(c, TM_EINVAL, "n1=%d n2=%d: both must be powers of two >= 1", d.n1, d.n2);
  if (d.K < 1 || d.K > 64) return fail(c, TM_EINVAL, "K=%d outside 1..64", d.K);
  if (d.P < 0) return fail(c, TM_EINVAL, "P=%d < 0", d.P);
  if ((int64_t)d.n1 * d.n2 > TW_MAX) return fail(c, TM_EUNSUPPORTED, "N=%d > %d", d.n1 * d.n2, TW_MAX);
  int L1 = ilog2(d.n1), L2 = ilog2(d.n2);
  auto v = c->variant.find((L1 << 8) | L2);
  *fn = tmk::find_row_launcher(L1, L2, v == c->variant.end() ? 0 : v->second);
  if (!*fn) return fail(c, TM_EUNSUPPORTED, "grid %dx%d has no compiled FFT plan", d.n1, d.n2);
  return TM_OK;
}

// The first of two or more cyclic sweeps forms the Lanczos start's Ritz vector
// itself (from the basis rows and the Ritz coefficients): its projections do
// not depend on the row's scale, so the separate combination and rescaling
// passes are skipped. With one sweep the last sweep's sums would see the
// unscaled row, so the combination stays separate.
bool ritz_in_sweep(const tm_retrieve_opts& o) {
  return o.method == TM_METHOD_ER_CYCLIC && o.iters >= 2 &&
         (o.start == TM_START_LANCZOS || o.start == TM_START_LEARNED);
}

tmk::RowArgs base_args(tm_ctx* c, const tm_dims& d, const tm_c32* masks) {
  tmk::RowArgs a;
  memset(&a, 0, sizeof a);
  a.P = d.P;
  a.K = d.K;
  a.masks = (const tmk::cx<float>*)masks;
  a.tw32 = c->tw32;
  a.tw64 = c->tw64;
  return a;
}

hipEvent_t ev_get(tm_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

// Fold finished event pairs into the per-mode totals (synchronises them).
void prof_drain(tm_ctx* c) {
  for (auto& r : c->recs) {
    hipEventSynchronize(r.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess && r.mode >= 0 && r.mode < TM_PROF_MODES) {
      c->acc_ms[r.mode] += ms;
      c->acc_n[r.mode] += 1;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
}

int run_row(tm_ctx* c, tmk::row_launcher fn, int mode, int ibf16, const tmk::RowArgs& a, void* s) {
  hipEvent_t ea = nullptr, eb = nullptr;
  if (c->prof && a.P > 0) {
    if (c->recs.size() > 4096) prof_drain(c);
    ea = ev_get(c);
    eb = ev_get(c);
    hipEventRecord(ea, (hipStream_t)s);
  }
  int e = fn(mode, ibf16, a, s);
  if (ea) {
    hipEventRecord(eb, (hipStream_t)s);
    c->recs.push_back({mode, ea, eb});
  }
  if (e) return hipfail(c, e, "row kernel launch");
  return TM_OK;
}

// Event timing of the L-BFGS kernels (run_lbfgs calls these around its launches).
void lb_prof_begin(void* user, int mode, void* stream) {
  tm_ctx* c = (tm_ctx*)user;
  if (!c->prof) return;
  if (c->recs.size() > 4096) prof_drain(c);
  hipEvent_t ea = ev_get(c), eb = ev_get(c);
  hipEventRecord(ea, (hipStream_t)stream);
  c->recs.push_back({mode, ea, eb});
}
void lb_prof_end(void* user, int mode, void* stream) {
  tm_ctx* c = (tm_ctx*)user;
  if (!c->prof || c->recs.empty() || c->recs.back().mode != mode) return;
  hipEventRecord(c->recs.back().b, (hipStream_t)stream);
}

}  // namespace

extern "C" {

int tm_grid_supported(int32_t n1, int32_t n2) {
  if (!is_pow2(n1) || !is_pow2(n2) || (int64_t)n1 * n2 > TW_MAX) return 0;
  return tmk::find_row_launcher(ilog2(n1), ilog2(n2)) ? 1 : 0;
}

int tm_create(tm_ctx** out, int device) {
  if (!out) return fail(nullptr, TM_EINVAL, "ctx pointer is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(nullptr, TM_EHIP, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(nullptr, TM_EINVAL, "device %d of %d", device, ndev);
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, TM_EHIP, "hipSetDevice(%d) failed", device);
  if (device >= NA_MAX_DEVICES) return fail(nullptr, TM_EINVAL, "device %d >= %d", device, NA_MAX_DEVICES);
  void* sp = nullptr;
  {
    // once per device, with that device current: the device's own address of `scratch`
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
      hipError_t se = hipGetSymbolAddress(&g_scratch_ptr[device], HIP_SYMBOL(scratch));
      if (se != hipSuccess || !g_scratch_ptr[device]) {
        g_scratch_ptr[device] = nullptr;
        return fail(nullptr, TM_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(se));
      }
    }
    sp = g_scratch_ptr[device];
  }
  tm_ctx* c = new tm_ctx;
  c->device = device;
  c->scratch = sp;
  // Twiddle tables W_L^i = exp(-2 pi j i / L) for every power of two L <= TW_MAX,
  // the table of length L at offset L - 1; FP64 values, FP32 rounded once.
  std::vector<tmk::cx<double>> h64(2 * TW_MAX);
  std::vector<tmk::cx<float>> h32(2 * TW_MAX);
  for (int L = 1; L <= TW_MAX; L <<= 1) {
    for (int i = 0; i < L; ++i) {
      double ang = -2.0 * M_PI * ((double)i / (double)L);
      tmk::cx<double> w{std::cos(ang), std::sin(ang)};
      h64[L - 1 + i] = w;
      h32[L - 1 + i] = tmk::cx<float>{(float)w.x, (float)w.y};
    }
  }
  if (hipMalloc(&c->tw32, h32.size() * sizeof(h32[0])) != hipSuccess ||
      hipMalloc(&c->tw64, h64.size() * sizeof(h64[0])) != hipSuccess ||
      hipMemcpy(c->tw32, h32.data(), h32.size() * sizeof(h32[0]), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->tw64, h64.data(), h64.size() * sizeof(h64[0]), hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(c->tw32);
    hipFree(c->tw64);
    delete c;
    return fail(nullptr, TM_EHIP, "twiddle table upload failed");
  }
  *out = c;
  return TM_OK;
}

int tm_destroy(tm_ctx* c) {
  if (!c) return TM_EINVAL;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  prof_drain(c);
  for (auto e : c->pool) hipEventDestroy(e);
  if (c->pinned) hipHostFree(c->pinned);
  phase_graph_release(c);
  for (auto& kv : c->ws) hipFree(kv.second.p);
  hipFree(c->tw32);
  hipFree(c->tw64);
  delete c;
  return TM_OK;
}

const char* tm_last_error(const tm_ctx* c) {
  if (!c) return g_create_err.c_str();
  return c->err.c_str();
}

int tm_forward(tm_ctx* c, tm_dims d, const tm_c32* masks, const tm_c32* t, int out_kind,
               int out_dtype, void* out, void* stream) {
  if (!c) return TM_EINVAL;
  tmk::row_launcher fn;
  int r = check_dims(c, d, &fn);
  if (r) return r;
  if (d.P == 0) return TM_OK;
  if (!masks || !t || !out) return fail(c, TM_EINVAL, "null pointer argument");
  if (out_kind != TM_FIELD && out_kind != TM_INTENSITY) return fail(c, TM_EINVAL, "out_kind %d", out_kind);
  if (out_kind == TM_INTENSITY && out_dtype != TM_F32 && out_dtype != TM_BF16)
    return fail(c, TM_EINVAL, "out_dtype %d", out_dtype);
  HIPCHK(c, hipSetDevice(c->device));
  tmk::RowArgs a = base_args(c, d, masks);
  a.tin = (const tmk::cx<float>*)t;
  a.yout = out;
  a.out_bf16 = (out_dtype == TM_BF16);
  return run_row(c, fn, out_kind == TM_FIELD ? tmk::M_FWD_FIELD : tmk::M_FWD_INT, 0, a, stream);
}

int tm_adjoint(tm_ctx* c, tm_dims d, const tm_c32* masks, const tm_c32* y, tm_c32* x, void* stream) {
  if (!c) return TM_EINVAL;
  tmk::row_launcher fn;
  int r = check_dims(c, d, &fn);
  if (r) return r;
  if (d.P == 0) return TM_OK;
  if (!masks || !y || !x) return fail(c, TM_EINVAL, "null pointer argument");
  HIPCHK(c, hipSetDevice(c->device));
  tmk::RowArgs a = base_args(c, d, masks);
  a.yin = (const tmk::cx<float>*)y;
  a.tout = (tmk::cx<float>*)x;
  return run_row(c, fn, tmk::M_ADJ, 0, a, stream);
}

static int gradient_mode(tm_ctx* c, int mode, tm_dims d, const tm_c32* masks, const void* I, int I_dtype,
                         const tm_c32* t, tm_c32* grad, float* f, void* stream);

int tm_gradient(tm_ctx* c, tm_dims d, const tm_c32* masks, const void* I, int I_dtype,
                const tm_c32* t, tm_c32* grad, float* f, void* stream) {
  return gradient_mode(c, tmk::M_GRAD, d, masks, I, I_dtype, t, grad, f, stream);
}

int tm_amp_gradient(tm_ctx* c, tm_dims d, const tm_c32* masks, const void* I, int I_dtype,
                    const tm_c32* t, tm_c32* grad, float* f, void* stream) {
  return gradient_mode(c, tmk::M_AGRAD, d, masks, I, I_dtype, t, grad, f, stream);
}

static int gradient_mode(tm_ctx* c, int mode, tm_dims d, const tm_c32* masks, const void* I, int I_dtype,
                         const tm_c32* t, tm_c32* grad, float* f, void* stream) {
  if (!c) return TM_EINVAL;
  tmk::row_launcher fn;
  int r = check_dims(c, d, &fn);
  if (r) return r;
  if (d.P == 0) return TM_OK;
  if (!masks || !I || !t || !grad) return fail(c, TM_EINVAL, "null pointer argument");
  if (I_dtype != TM_F32 && I_dtype != TM_BF16) return fail(c, TM_EINVAL, "I_dtype %d", I_dtype);
  HIPCHK(c, hipSetDevice(c->device));
  float* sums = (float*)ws_get(c, WS_SUMS, (size_t)d.P * tmk::NSUM * sizeof(float));
  if (!sums) return fail(c, TM_ENOMEM, "workspace");
  tmk::RowArgs a = base_args(c, d, masks);
  a.I = I;
  a.tin = (const tmk::cx<float>*)t;
  a.tout = (tmk::cx<float>*)grad;
  a.sums = sums;
  r = run_row(c, fn, mode, I_dtype == TM_BF16, a, stream);
  if (r) return r;
  if (f) {
    HIPCHK(c, hipMemcpy2DAsync(f, sizeof(float), sums, tmk::NSUM * sizeof(float), sizeof(float), d.P,
                               hipMemcpyDeviceToDevice, (hipStream_t)stream));
  }
  return TM_OK;
}

static int residual_into(tm_ctx* c, tmk::row_launcher fn, const tm_dims& d, const tm_c32* masks,
                         const void* I, int I_dtype, const tm_c32* t, double* sums64, void* stream) {
  tmk::RowArgs a = base_args(c, d, masks);
  a.I = I;
  a.tin = (const tmk::cx<float>*)t;
  a.sums64 = sums64;
  return run_row(c, fn, tmk::M_RES64, I_dtype == TM_BF16, a, stream);
}

int tm_residual_f64(tm_ctx* c, tm_dims d, const tm_c32* masks, const void* I, int I_dtype,
                    const tm_c32* t, double* rho, void* stream) {
  if (!c) return TM_EINVAL;
  tmk::row_launcher fn;
  int r = check_dims(c, d, &fn);
  if (r) return r;
  if (d.P == 0) return TM_OK;
  if (!masks || !I || !t || !rho) return fail(c, TM_EINVAL, "null pointer argument");
  if (I_dtype != TM_F32 && I_dtype != TM_BF16) return fail(c, TM_EINVAL, "I_dtype %d", I_dtype);
  HIPCHK(c, hipSetDevice(c->device));
  double* s64 = (double*)ws_get(c, WS_SUMS64, (size_t)d.P * 2 * sizeof(double));
  void* st = ws_get(c, WS_LB_ST, (size_t)d.P * sizeof(tm_row_stats));
  if (!s64 || !st) return fail(c, TM_ENOMEM, "workspace");
  r = residual_into(c, fn, d, masks, I, I_dtype, t, s64, stream);
  if (r) return r;
  int e = tmk::launch_finalize(st, d.P, s64, nullptr, 0, -1, -1, 0, 1e-2, stream);
  if (e) return hipfail(c, e, "finalize");
  HIPCHK(c, hipMemcpy2DAsync(rho, sizeof(double), st, sizeof(tm_row_stats), sizeof(double), d.P,
                             hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return TM_OK;
}

int tm_retrieve(tm_ctx* c, tm_dims d, const tm_c32* masks, const void* I, tm_c32* t,
                const tm_retrieve_opts* o, tm_row_stats* stats, void* stream) {
  if (!c) return TM_EINVAL;
  tmk::row_launcher fn;
  int r = check_dims(c, d, &fn);
  if (r) return r;
  if (!o) return fail(c, TM_EINVAL, "opts is NULL");
  if (o->method != TM_METHOD_ER && o->method != TM_METHOD_LBFGS && o->method != TM_METHOD_LBFGS_AMP &&
      o->method != TM_METHOD_ER_CYCLIC)
    return fail(c, TM_EINVAL, "method %d", o->method);
  const bool er_like = o->method == TM_METHOD_ER || o->method == TM_METHOD_ER_CYCLIC;
  if (o->iters < 0) return fail(c, TM_EINVAL, "iters %d < 0", o->iters);
  if (o->I_dtype != TM_F32 && o->I_dtype != TM_BF16) return fail(c, TM_EINVAL, "I_dtype %d", o->I_dtype);
  if (o->start < TM_START_GIVEN || o->start > TM_START_LEARNED) return fail(c, TM_EINVAL, "start %d", o->start);
  if (o->start == TM_START_LEARNED && c->wtab_n < 2)
    return fail(c, TM_EINVAL, "TM_START_LEARNED needs a weight table (tm_set_weight_table)");
  if (o->start == TM_START_LANCZOS || o->start == TM_START_LEARNED) {
    if (o->spectral_iters < 1 || o->spectral_iters > tmk::LZ_MAX)
      return fail(c, TM_EINVAL, "Lanczos steps (spectral_iters) %d outside 1..%d", o->spectral_iters, tmk::LZ_MAX);
    if (!(o->spectral_tau > 0.f)) return fail(c, TM_EINVAL, "spectral_tau must be > 0");
  }
  if (o->start == TM_START_SPECTRAL) {
    if (o->spectral_iters < 0) return fail(c, TM_EINVAL, "spectral_iters %d", o->spectral_iters);
    if (!(o->spectral_tau > 0.f)) return fail(c, TM_EINVAL, "spectral_tau must be > 0");
    if (!(o->spectral_momentum >= 0.f && o->spectral_momentum < 1.f))
      return fail(c, TM_EINVAL, "spectral_momentum must be in [0, 1)");
    if (!(o->spectral_lower >= -1.f && o->spectral_lower <= o->spectral_momentum))
      return fail(c, TM_EINVAL, "spectral_lower must be in [-1, spectral_momentum]");
  }
  if (!(o->er_momentum >= 0.f && o->er_momentum < 1.f)) return fail(c, TM_EINVAL, "er_momentum must be in [0, 1)");
  if (o->method == TM_METHOD_ER_CYCLIC && o->er_momentum != 0.f)
    return fail(c, TM_EINVAL, "cyclic error reduction takes no momentum (er_momentum must be 0)");
  if (!er_like && (o->lbfgs_m < 1 || o->lbfgs_m > 16))
    return fail(c, TM_EINVAL, "lbfgs_m %d outside 1..16", o->lbfgs_m);
  if (d.P == 0) return TM_OK;
  if (!masks || !I || !t) return fail(c, TM_EINVAL, "null pointer argument");
  HIPCHK(c, hipSetDevice(c->device));
  const int N = d.n1 * d.n2;
  const int ibf = o->I_dtype == TM_BF16;
  float* sums = (float*)ws_get(c, WS_SUMS, (size_t)d.P * tmk::NSUM * sizeof(float));
  double* s64 = (double*)ws_get(c, WS_SUMS64, (size_t)d.P * 2 * sizeof(double));
  if (!sums || !s64) return fail(c, TM_ENOMEM, "workspace");
  tmk::RowArgs a = base_args(c, d, masks);
  a.I = I;
  tmk::cx<float>* tt = (tmk::cx<float>*)t;
  const tmk::cx<float>* ritz_basis = nullptr;  // Lanczos basis and Ritz coefficients for the first sweep
  const double* ritz_y = nullptr;
  int ritz_k = 0;

  // ---- start
  if (o->start == TM_START_BACKPROP) {
    a.tout = tt;
    r = run_row(c, fn, tmk::M_BACKPROP, ibf, a, stream);
    if (r) return r;
  } else if (o->start == TM_START_SPECTRAL) {
    double* rowsum = (double*)ws_get(c, WS_ROWSUM, (size_t)d.P * sizeof(double));
    float* rowmean = (float*)ws_get(c, WS_ROWMEAN, (size_t)d.P * sizeof(float));
    void* vprev = ws_get(c, WS_VPREV, (size_t)d.P * N * sizeof(tm_c32));
    float* vscale = (float*)ws_get(c, WS_VSCALE, (size_t)d.P * sizeof(float));
    if (!rowsum || !rowmean || !vprev || !vscale) return fail(c, TM_ENOMEM, "workspace");
    int e = tmk::launch_row_isum(I, ibf, (int64_t)d.K * N, d.P, rowsum, rowmean, stream);
    if (!e) e = tmk::launch_row_rescale(t, N, d.P, 0, nullptr, 1.0, stream);
    if (!e) e = tmk::launch_fill_zero(vprev, (int64_t)d.P * N * sizeof(tm_c32), stream);
    if (!e) e = tmk::launch_fill_zero(vscale, (int64_t)d.P * sizeof(float), stream);
    if (e) return hipfail(c, e, "spectral setup");
    // v and the previous iterate alternate between t and the workspace row buffer
    tmk::cx<float>* vb[2] = {tt, (tmk::cx<float>*)vprev};
    tmk::RowArgs s = a;
    s.rowmean = rowmean;
    s.vscale = vscale;
    s.tau = o->spectral_tau;
    s.momentum = o->spectral_momentum;
    s.spec_lower = o->spectral_lower;
    s.sums = sums;
    for (int it = 0; it < o->spectral_iters; ++it) {
      s.tin = vb[it & 1];
      s.din = vb[(it & 1) ^ 1];
      s.tout = vb[(it & 1) ^ 1];
      r = run_row(c, fn, tmk::M_SPEC, ibf, s, stream);
      if (r) return r;
    }
    if (o->spectral_iters & 1) e = tmk::launch_copy(t, vprev, (int64_t)d.P * N * sizeof(tm_c32), stream);
    if (!e) e = tmk::launch_row_rescale(t, N, d.P, 1, rowsum, (double)d.K * N, stream);
    if (e) return hipfail(c, e, "spectral scale");
  } else if (o->start == TM_START_LANCZOS || o->start == TM_START_LEARNED) {
    // v_1 = seed / ||seed|| in t; v_2 .. v_{k+1} in the workspace; (alpha, beta) per step and row
    const int k = o->spectral_iters;
    const size_t rowsz = (size_t)d.P * N;
    double* rowsum = (double*)ws_get(c, WS_ROWSUM, (size_t)d.P * sizeof(double));
    float* rowmean = (float*)ws_get(c, WS_ROWMEAN, (size_t)d.P * sizeof(float));
    tmk::cx<float>* Vw = (tmk::cx<float>*)ws_get(c, WS_LZ_V, (size_t)k * rowsz * sizeof(tm_c32));
    float* hist = (float*)ws_get(c, WS_LZ_H, (size_t)k * d.P * 2 * sizeof(float));
    double* y = (double*)ws_get(c, WS_LZ_Y, (size_t)k * d.P * sizeof(double));
    if (!rowsum || !rowmean || !Vw || !hist || !y) return fail(c, TM_ENOMEM, "Lanczos workspace");
    const bool learned = o->start == TM_START_LEARNED;
    int e = 0;
    if (learned) {  // the weights need the row means before the first step; otherwise that step forms them
      e = tmk::launch_row_isum(I, ibf, (int64_t)d.K * N, d.P, rowsum, rowmean, stream);
      if (!e) e = tmk::launch_row_rescale(t, N, d.P, 0, nullptr, 1.0, stream);
      if (e) return hipfail(c, e, "Lanczos setup");
    }
    auto V = [&](int j) { return j == 0 ? tt : Vw + (size_t)(j - 1) * rowsz; };
    tmk::RowArgs s = a;
    s.rowmean = rowmean;
    s.tau = o->spectral_tau;
    if (learned) {
      // the learned weights of every measurement, evaluated once: the Lanczos
      // steps then read them in place of the intensities (same bytes as FP32 I)
      float* W = (float*)ws_get(c, WS_PH_BASE + 47, (size_t)d.P * d.K * N * sizeof(float));
      const float* tab = (const float*)ws_get(c, WS_WTAB, (size_t)c->wtab_n * 2 * sizeof(float));
      if (!W || !tab) return fail(c, TM_ENOMEM, "learned weight workspace");
      e = tmk::wnet_weights(I, ibf, rowmean, d.P, (int64_t)d.K * N, tab, c->wtab_n, c->wtab_xmax, W, stream);
      if (e) return hipfail(c, e, "learned weights");
      s.I = W;
    }
    for (int j = 0; j < k; ++j) {
      s.tin = V(j);
      s.din = V(j > 0 ? j - 1 : 0);
      s.tout = V(j + 1);
      s.lz_bprev = j > 0 ? hist + (size_t)(j - 1) * d.P * 2 : nullptr;
      s.lz_out = hist + (size_t)j * d.P * 2;
      s.lz_sum = (!learned && j == 0) ? rowsum : nullptr;  // the first step: row sums, means, unit seed
      s.lz_mean = (!learned && j == 0) ? rowmean : nullptr;
      r = run_row(c, fn, learned ? tmk::M_LANCZOS_T : tmk::M_LANCZOS, learned ? 0 : ibf, s, stream);
      if (r) return r;
    }
    e = tmk::launch_lz_ritz(hist, k, d.P, y, stream);
    if (!e && !ritz_in_sweep(*o)) e = tmk::launch_lz_combine_scaled(t, Vw, y, k, d.P, N, rowsum, (double)d.K * N, stream);
    if (e) return hipfail(c, e, "Lanczos Ritz vector");
    if (ritz_in_sweep(*o)) {  // the first cyclic sweep forms the Ritz vector (its scale does not matter there)
      ritz_basis = Vw;
      ritz_y = y;
      ritz_k = k;
    }
  }

  // ---- iterations
  int f_idx = -1, amp_idx = -1;
  if (o->method == TM_METHOD_ER_CYCLIC) {
    a.tin = tt;
    a.tout = tt;
    for (int it = 0; it < o->iters; ++it) {
      a.sums = (it == o->iters - 1) ? sums : nullptr;  // only the last sweep's sums are reported
      tmk::RowArgs s = a;
      if (it == 0 && ritz_k > 0) {
        s.lz_basis = ritz_basis;
        s.lz_y = ritz_y;
        s.lz_k = ritz_k;
        s.lz_rs = (int64_t)d.P * N;
      }
      r = run_row(c, fn, tmk::M_ERC, ibf, s, stream);
      if (r) return r;
    }
    if (o->iters > 0) {
      amp_idx = 0;
      f_idx = 1;
    }
  } else if (o->method == TM_METHOD_ER) {
    a.tin = tt;
    a.tout = tt;
    const bool mom = o->er_momentum > 0.f && o->iters > 0;
    tmk::cx<float>* buf[2] = {tt, nullptr};
    if (mom) {
      // t_prev starts equal to t; t and t_prev then alternate between the
      // caller's buffer and the workspace (the new iterate overwrites t_prev)
      buf[1] = (tmk::cx<float>*)ws_get(c, WS_TPREV, (size_t)d.P * N * sizeof(tm_c32));
      if (!buf[1]) return fail(c, TM_ENOMEM, "workspace");
      int ce = tmk::launch_copy(buf[1], t, (int64_t)d.P * N * sizeof(tm_c32), stream);
      if (ce) return hipfail(c, ce, "momentum copy");
      a.er_beta = o->er_momentum;
    }
    for (int it = 0; it < o->iters; ++it) {
      a.sums = (it == o->iters - 1) ? sums : nullptr;  // only the last iteration's sums are reported
      if (mom) {
        a.tin = buf[it & 1];
        a.din = buf[(it & 1) ^ 1];
        a.tout = buf[(it & 1) ^ 1];
      }
      r = run_row(c, fn, tmk::M_ER, ibf, a, stream);
      if (r) return r;
    }
    if (mom && (o->iters & 1)) {
      int ce = tmk::launch_copy(t, buf[1], (int64_t)d.P * N * sizeof(tm_c32), stream);
      if (ce) return hipfail(c, ce, "momentum copy");
    }
    if (o->iters > 0) {
      amp_idx = 0;
      f_idx = 1;
    }
  } else {
    tmk::LbfgsBuffers b;
    size_t vec = (size_t)d.P * N * sizeof(tm_c32);
    b.g = ws_get(c, WS_LB_G, vec);
    b.gp = ws_get(c, WS_LB_GP, vec);
    b.d = ws_get(c, WS_LB_D, vec);
    b.S = ws_get(c, WS_LB_S, vec * tmk::LB_SLOTS(o->lbfgs_m));
    b.Y = ws_get(c, WS_LB_Y, vec * tmk::LB_SLOTS(o->lbfgs_m));
    b.sc = ws_get(c, WS_LB_SC, (size_t)d.P * tmk::LB_SCALARS(o->lbfgs_m) * sizeof(double));
    b.dots = ws_get(c, WS_PH_BASE + 48, (size_t)d.P * tmk::LB_DOTS(N) * sizeof(double));
    if (!b.g || !b.gp || !b.d || !b.S || !b.Y || !b.sc || !b.dots) return fail(c, TM_ENOMEM, "L-BFGS workspace");
    b.sums = sums;
    b.hook_user = c;
    b.hook_begin = lb_prof_begin;
    b.hook_end = lb_prof_end;
    const int amp = o->method == TM_METHOD_LBFGS_AMP;
    int e = tmk::run_lbfgs(fn, a, ibf, N, o->iters, o->lbfgs_m, tt, b, stream, amp);
    if (e) return hipfail(c, e, "L-BFGS");
    if (amp) amp_idx = 0;  // the amplitude cost sum (sqrt(I) - |A t|)^2
    else f_idx = 0;
  }

  // ---- FP64 acceptance residual and per-row record
  r = residual_into(c, fn, d, masks, I, o->I_dtype, t, s64, stream);
  if (r) return r;
  if (stats) {
    int e = tmk::launch_finalize(stats, d.P, s64, (f_idx >= 0 || amp_idx >= 0) ? sums : nullptr, tmk::NSUM, f_idx,
                                 amp_idx, o->iters, 1e-2, stream);
    if (e) return hipfail(c, e, "finalize");
  }
  return TM_OK;
}

int tm_retrieve_noalloc(tm_ctx* c, tm_dims d, const tm_c32* masks, const void* I, tm_c32* t,
                        const tm_retrieve_opts* o, tm_row_stats* stats, void* stream) {
  if (!c) return TM_EINVAL;
  tmk::row_launcher fn;
  int r = check_dims(c, d, &fn);
  if (r) return r;
  if (!o) return fail(c, TM_EINVAL, "opts is NULL");
  if (o->method != TM_METHOD_ER && o->method != TM_METHOD_ER_CYCLIC)
    return fail(c, TM_EUNSUPPORTED, "method %d: the allocation-free form runs TM_METHOD_ER or TM_METHOD_ER_CYCLIC",
                o->method);
  if (o->start != TM_START_GIVEN && o->start != TM_START_BACKPROP)
    return fail(c, TM_EUNSUPPORTED, "start %d: the allocation-free form starts from TM_START_GIVEN or "
                "TM_START_BACKPROP", o->start);
  if (o->er_momentum != 0.f) return fail(c, TM_EUNSUPPORTED, "er_momentum: the allocation-free form takes none");
  if (o->iters < 0) return fail(c, TM_EINVAL, "iters %d < 0", o->iters);
  if (o->I_dtype != TM_F32 && o->I_dtype != TM_BF16) return fail(c, TM_EINVAL, "I_dtype %d", o->I_dtype);
  if (d.P > TM_NOALLOC_MAX_ROWS)
    return fail(c, TM_EINVAL, "P=%d exceeds the allocation-free limit of %d rows", d.P, TM_NOALLOC_MAX_ROWS);
  if (d.P == 0) return TM_OK;
  if (!masks || !I || !t) return fail(c, TM_EINVAL, "null pointer argument");
  if (!c->scratch) return fail(c, TM_EHIP, "no scratch address for device %d", c->device);
  HIPCHK(c, hipSetDevice(c->device));
  // every value read from the scratch is written earlier in this call (sums
  // and residual sums are stored per row, not accumulated)
  float* sums = (float*)c->scratch;
  double* s64 = (double*)((unsigned char*)c->scratch + NA_S64_OFF);
  const int ibf = o->I_dtype == TM_BF16;
  tmk::RowArgs a = base_args(c, d, masks);
  a.I = I;
  tmk::cx<float>* tt = (tmk::cx<float>*)t;
  int e = 0;
  if (o->start == TM_START_BACKPROP) {
    a.tout = tt;
    e = fn(tmk::M_BACKPROP, ibf, a, stream);
    if (e) return hipfail(c, e, "row kernel launch");
  }
  const int mode = o->method == TM_METHOD_ER_CYCLIC ? tmk::M_ERC : tmk::M_ER;
  a.tin = tt;
  a.tout = tt;
  for (int it = 0; it < o->iters; ++it) {
    a.sums = (it == o->iters - 1) ? sums : nullptr;  // only the last iteration's sums are reported
    e = fn(mode, ibf, a, stream);
    if (e) return hipfail(c, e, "row kernel launch");
  }
  tmk::RowArgs ra = base_args(c, d, masks);
  ra.I = I;
  ra.tin = tt;
  ra.sums64 = s64;
  e = fn(tmk::M_RES64, ibf, ra, stream);
  if (e) return hipfail(c, e, "row kernel launch");
  if (stats) {
    const bool any = o->iters > 0;
    e = tmk::launch_finalize(stats, d.P, s64, any ? sums : nullptr, tmk::NSUM, any ? 1 : -1, any ? 0 : -1,
                             o->iters, 1e-2, stream);
    if (e) return hipfail(c, e, "finalize");
  }
  return TM_OK;
}

}  // extern "C"

// Argument checks of the phase entry points. host_pix: also read pix back and
// check its range and distinctness here (tm_phase_offset_correct checks it on
// the device instead, so that it does not wait for earlier work on the stream).
static int phase_check(tm_ctx* c, const tm_defocus_dims* dd, const int32_t* pix, const tm_c32* tm_est,
                       const tm_c32* theta, const float* I_d, const tm_optics* o, bool host_pix = true) {
  if (!dd || !o) return fail(c, TM_EINVAL, "dims/optics pointer is NULL");
  if (dd->P < 1 || dd->N < 1 || dd->Nd < 1) return fail(c, TM_EINVAL, "P=%d N=%d Nd=%d must be >= 1", dd->P, dd->N, dd->Nd);
  if (!is_pow2(dd->nf1) || !is_pow2(dd->nf2) || dd->nf1 < 2 || dd->nf2 < 2 || dd->nf1 > 256 || dd->nf2 > 256)
    return fail(c, TM_EINVAL, "field grid %dx%d: powers of two in 2..256", dd->nf1, dd->nf2);
  if ((int64_t)dd->P > (int64_t)dd->nf1 * dd->nf2) return fail(c, TM_EINVAL, "P=%d exceeds the field grid", dd->P);
  if (!pix || !tm_est || !theta || !I_d) return fail(c, TM_EINVAL, "null pointer argument");
  if (!(o->lambda > 0) || !(o->ps_field > 0) || !(o->NA > 0) || !(o->NA < 1) || !std::isfinite(o->z))
    return fail(c, TM_EINVAL, "optics: lambda, ps_field > 0, 0 < NA < 1, finite z");
  if (!host_pix) return TM_OK;
  // pixel indices address the field grid: check range and distinctness on the host
  std::vector<int32_t> hp(dd->P);
  if (hipMemcpy(hp.data(), pix, dd->P * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, TM_EHIP, "reading pix");
  std::vector<char> seen((size_t)dd->nf1 * dd->nf2, 0);
  for (int i = 0; i < dd->P; ++i) {
    if (hp[i] < 0 || hp[i] >= dd->nf1 * dd->nf2) return fail(c, TM_EINVAL, "pix[%d]=%d outside the field grid", i, hp[i]);
    if (seen[hp[i]]) return fail(c, TM_EINVAL, "pix[%d]=%d repeats a pixel", i, hp[i]);
    seen[hp[i]] = 1;
  }
  return TM_OK;
}

static int phase_prepare(tm_ctx* c, const tm_defocus_dims* dd, const int32_t* pix, const tm_c32* tm_est,
                         const tm_c32* theta, const tm_optics* o, tmk::PhaseDims& pd, tmk::PhaseWork& w,
                         void* stream) {
  pd = tmk::PhaseDims{dd->P, dd->N, dd->Nd, dd->nf1, dd->nf2};
  void* base = ws_get(c, WS_PH_BASE, tmk::phase_work_bytes(pd));
  if (!base) return fail(c, TM_ENOMEM, "phase workspace");
  tmk::phase_work_carve(base, pd, &w);
  tmk::PhaseOptics po{o->lambda, o->ps_field, o->NA, o->z};
  w.band = tmk::phase_band_plan(pd, po, c->phase_band);
  int e = tmk::phase_setup(pd, po, tm_est, theta, pix, w, stream);
  if (e) return hipfail(c, e, "phase setup");
  // c[n][p] = sum_k theta[n][k] tm_est[p][k] in FP64 (exact products of the FP32 inputs)
  double* part = (double*)ws_get(c, WS_PH_BASE + 2,
                                 (size_t)tmk::phase_cgemm_slices(pd) * dd->Nd * dd->P * 2 * sizeof(double));
  if (!part) return fail(c, TM_ENOMEM, "phase GEMM workspace");
  e = tmk::phase_cgemm(pd, theta, tm_est, part, w.c, stream);
  if (e) return hipfail(c, e, "phase GEMM");
  return TM_OK;
}

extern "C" int tm_phase_set_band(tm_ctx* c, int32_t enable) {
  if (!c) return TM_EINVAL;
  if (enable != 0 && enable != 1) return fail(c, TM_EINVAL, "enable must be 0 or 1");
  c->phase_band = enable;
  return TM_OK;
}

extern "C" int tm_phase_objective(tm_ctx* c, const tm_defocus_dims* dd, const int32_t* pix, const tm_c32* tm_est,
                                  const tm_c32* theta, const float* I_d, const tm_optics* o, const double* phi,
                                  double* g_dev, double* grad, void* stream) {
  if (!c) return TM_EINVAL;
  int r = phase_check(c, dd, pix, tm_est, theta, I_d, o);
  if (r) return r;
  if (!phi || !g_dev || !grad) return fail(c, TM_EINVAL, "null pointer argument");
  HIPCHK(c, hipSetDevice(c->device));
  tmk::PhaseDims pd;
  tmk::PhaseWork w;
  if ((r = phase_prepare(c, dd, pix, tm_est, theta, o, pd, w, stream))) return r;
  int e = tmk::phase_eval(pd, pix, I_d, phi, grad, w, (const double*)c->tw64, stream);
  if (e) return hipfail(c, e, "phase eval");
  HIPCHK(c, hipMemcpyAsync(g_dev, w.gval, sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return TM_OK;
}

// Graph iterations the solve may take: at most 40 trials per accepted
// iteration, plus the iteration that decides the last trial and ends it.
static long phase_max_evals(int iters) { return (long)iters * 40 + 2; }

// The phase solve of tm_phase_offset_correct (rec_dev == NULL: batches of
// graph replays until the device state says the solve has ended, the host
// reading that state between batches) and of tm_phase_offset_correct_async
// (rec_dev != NULL: `evals` graph iterations queued, the end-of-solve record
// written to rec_dev, no wait).
static int phase_solve(tm_ctx* c, const tm_defocus_dims* dd, const int32_t* pix, const tm_c32* tm_est,
                       const tm_c32* theta, const float* I_d, const tm_optics* o, double* phi,
                       const tm_phase_opts* po, double* g_out, void* stream, long evals, double* rec_dev) {
  if (!c) return TM_EINVAL;
  int r = phase_check(c, dd, pix, tm_est, theta, I_d, o, false);
  if (r) return r;
  if (!phi || !po) return fail(c, TM_EINVAL, "null pointer argument");
  if (po->iters < 0 || po->m < 1 || po->m > 16) return fail(c, TM_EINVAL, "iters >= 0 and 1 <= m <= 16");
  if (!(po->ftol >= 0.0)) return fail(c, TM_EINVAL, "ftol must be >= 0");
  const bool async = rec_dev != nullptr;
  if (async && po->iters > 0 && (evals < 1 || evals > phase_max_evals(po->iters)))
    return fail(c, TM_EINVAL, "evals=%ld outside 1..%ld", evals, phase_max_evals(po->iters));
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  tmk::PhaseDims pd;
  tmk::PhaseWork w;
  if ((r = phase_prepare(c, dd, pix, tm_est, theta, o, pd, w, stream))) return r;
  const int P = dd->P, m = po->m;
  size_t vb = ((P * sizeof(double) + 255) / 256) * 256;
  char* lb = (char*)ws_get(c, WS_PH_BASE + 1,
                          vb * (6 + 2 * m) + (tmk::phase_lb_state_doubles(m) + 8) * sizeof(double));
  if (!lb) return fail(c, TM_ENOMEM, "phase L-BFGS workspace");
  tmk::PhaseLb L;
  L.phi = (double*)(lb);
  L.g = (double*)(lb + vb);
  L.gt = (double*)(lb + 2 * vb);
  L.phit = (double*)(lb + 3 * vb);
  L.d = (double*)(lb + 4 * vb);
  L.gb = (double*)(lb + 5 * vb);
  L.S = (double*)(lb + 6 * vb);
  L.Y = (double*)(lb + (6 + m) * vb);
  L.sc = (double*)(lb + (6 + 2 * m) * vb);
  L.dpart = w.dpart;
  double* rec = L.sc + tmk::phase_lb_state_doubles(m);  // 8 doubles: the end-of-batch record
  HIPCHK(c, hipMemcpyAsync(L.phi, phi, P * sizeof(double), hipMemcpyDeviceToDevice, s));
  int e = tmk::phase_eval(pd, pix, I_d, L.phi, L.g, w, (const double*)c->tw64, stream);
  if (!e) e = tmk::phase_lb_init(L, P, m, po->iters, w.gval, w.skip, w.chk, stream);
  if (e) return hipfail(c, e, "phase start");
  if (!async && !c->pinned) HIPCHK(c, hipHostMalloc((void**)&c->pinned, 8 * sizeof(double), hipHostMallocDefault));
  double* hb = c->pinned;
  // end of a batch: phi out (device-side, skipped after a failed pixel check)
  // and the record (f, iterations, evaluations, ended, pixel check) read back
  auto finish = [&]() -> int {
    int fe = tmk::phase_lb_finish(L, w, P, phi, rec, stream);
    hipError_t fh = fe ? hipSuccess : hipMemcpyAsync(hb, rec, 7 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (!fe && fh == hipSuccess) fh = hipStreamSynchronize(s);
    return fe ? fe : (int)fh;
  };
  // One iteration (decision on the pending trial, new direction or changed
  // step, trial point, objective and gradient there) is a captured graph; the line-search
  // control lives in device state, so replays are queued back-to-back and
  // the host reads the state only between batches of replays.
  if (po->iters > 0) {
    // everything the captured iteration depends on
    const tmk::PhaseBand& bd = w.band;
    std::vector<double> key = {(double)pd.P, (double)pd.N, (double)pd.Nd, (double)pd.nf1, (double)pd.nf2,
                               (double)(uintptr_t)pix, (double)(uintptr_t)I_d, (double)(uintptr_t)lb,
                               (double)(uintptr_t)w.c, (double)(uintptr_t)c->tw64, (double)m, (double)po->iters,
                               po->ftol, (double)bd.on, (double)bd.s1lo, (double)bd.B1, (double)bd.s2lo,
                               (double)bd.B2, (double)bd.RA, (double)bd.CH, (double)bd.G, (double)bd.CPW,
                               (double)bd.NXB, (double)c->device};
    if (!(c->pg.exec && c->pg.key == key)) {
      phase_graph_release(c);
      hipStream_t cap = nullptr;
      hipGraph_t graph = nullptr;
      hipGraphExec_t gexec = nullptr;
      hipError_t he = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
      if (he == hipSuccess) he = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
      if (he == hipSuccess) {
        // several iterations per replay, so that one launch from the host covers
        // them (an iteration after the solve has ended returns at once)
        for (int r = 0; r < PHASE_GRAPH_ITERS && !e; ++r) {
          e = tmk::phase_lb_iter(L, P, m, po->iters, po->ftol, w.gval, w.skip, cap);
          if (!e) e = tmk::phase_eval(pd, pix, I_d, L.phit, L.gt, w, (const double*)c->tw64, cap, L.d);
        }
        hipError_t he2 = hipStreamEndCapture(cap, &graph);
        if (!e && he2 == hipSuccess) he2 = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
        if (!e && he2 != hipSuccess) e = (int)he2;
      } else {
        e = (int)he;
      }
      c->pg.g = graph;
      c->pg.exec = gexec;
      c->pg.cap = cap;
      if (!e) c->pg.key = key;
      else phase_graph_release(c);
    }
    hipGraphExec_t gexec = c->pg.exec;
    if (async) {
      // whole replays, then the remaining iterations launched one by one (the same kernels)
      for (long i = 0; i < evals / PHASE_GRAPH_ITERS && !e; ++i) e = (int)hipGraphLaunch(gexec, s);
      for (long i = 0; i < evals % PHASE_GRAPH_ITERS && !e; ++i) {
        e = tmk::phase_lb_iter(L, P, m, po->iters, po->ftol, w.gval, w.skip, stream);
        if (!e) e = tmk::phase_eval(pd, pix, I_d, L.phit, L.gt, w, (const double*)c->tw64, stream, L.d);
      }
      if (!e) e = tmk::phase_lb_finish(L, w, P, phi, rec_dev, stream);
      if (e) return hipfail(c, e, "phase iterations");
      return TM_OK;
    }
    // PHASE_GRAPH_ITERS graph iterations per replay
    const long limit = (phase_max_evals(po->iters) + PHASE_GRAPH_ITERS - 1) / PHASE_GRAPH_ITERS;
    // first batch: enough replays for the evaluations the last solve of the same
    // iteration count took (every graph iteration but the last evaluates one
    // trial), else for one trial per iteration plus a margin
    const long guess = (c->ph_evals > 0 && c->ph_iters_req == po->iters) ? (long)c->ph_evals : (long)po->iters + 8;
    long launched = 0, batch = (guess + PHASE_GRAPH_ITERS - 1) / PHASE_GRAPH_ITERS;
    while (!e && launched < limit) {
      long nb = std::min(batch, limit - launched);
      for (long i = 0; i < nb && !e; ++i) e = (int)hipGraphLaunch(gexec, s);
      launched += nb;
      if (!e) e = finish();
      if (e || hb[3] != 0.0) break;  // error, or the solve has ended
      batch = 2;
    }
    if (e) return hipfail(c, e, "phase iterations");
  } else if (async) {
    e = tmk::phase_lb_finish(L, w, P, phi, rec_dev, stream);
    if (e) return hipfail(c, e, "phase result");
    return TM_OK;
  } else {
    e = finish();
    if (e) return hipfail(c, e, "phase result");
  }
  if (hb[4] != 0.0) {  // pixel check failed: phi is left as it was
    const bool range = ((int)hb[4] & 1) != 0;
    const int32_t bp = (int32_t)(range ? hb[5] : hb[6]);
    int32_t gv = -1;
    if (bp >= 0 && bp < P) HIPCHK(c, hipMemcpy(&gv, pix + bp, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (range) return fail(c, TM_EINVAL, "pix[%d]=%d outside the field grid", bp, gv);
    return fail(c, TM_EINVAL, "pix[%d]=%d repeats a pixel", bp, gv);
  }
  const double f = hb[0];
  c->ph_iters = (int32_t)hb[1];
  c->ph_evals = (int32_t)hb[2];
  c->ph_iters_req = po->iters;
  if (g_out) *g_out = f;
  return TM_OK;
}

extern "C" int tm_phase_offset_correct(tm_ctx* c, const tm_defocus_dims* dd, const int32_t* pix,
                                       const tm_c32* tm_est, const tm_c32* theta, const float* I_d,
                                       const tm_optics* o, double* phi, const tm_phase_opts* po,
                                       double* g_out, void* stream) {
  return phase_solve(c, dd, pix, tm_est, theta, I_d, o, phi, po, g_out, stream, 0, nullptr);
}

extern "C" int tm_phase_offset_correct_async(tm_ctx* c, const tm_defocus_dims* dd, const int32_t* pix,
                                             const tm_c32* tm_est, const tm_c32* theta, const float* I_d,
                                             const tm_optics* o, double* phi, const tm_phase_opts* po,
                                             int32_t evals, double* rec, void* stream) {
  if (!c) return TM_EINVAL;
  if (!rec) return fail(c, TM_EINVAL, "null pointer argument");
  return phase_solve(c, dd, pix, tm_est, theta, I_d, o, phi, po, nullptr, stream, evals, rec);
}

extern "C" int tm_phase_last_counts(tm_ctx* c, int32_t* iterations, int32_t* evaluations) {
  if (!c || !iterations || !evaluations) return TM_EINVAL;
  *iterations = c->ph_iters;
  *evaluations = c->ph_evals;
  return TM_OK;
}

extern "C" int tm_defocus_forward(tm_ctx* c, const tm_defocus_dims* dd, const int32_t* pix, const tm_c32* tmr,
                                  const tm_c32* theta, const tm_optics* o, const double* phi, float* I_out,
                                  void* stream) {
  if (!c) return TM_EINVAL;
  int r = phase_check(c, dd, pix, tmr, theta, I_out, o);
  if (r) return r;
  if (!phi) return fail(c, TM_EINVAL, "null pointer argument");
  HIPCHK(c, hipSetDevice(c->device));
  tmk::PhaseDims pd;
  tmk::PhaseWork w;
  if ((r = phase_prepare(c, dd, pix, tmr, theta, o, pd, w, stream))) return r;
  int e = tmk::phase_images(pd, pix, phi, I_out, w, (const double*)c->tw64, stream);
  if (e) return hipfail(c, e, "defocus images");
  return TM_OK;
}

extern "C" int tm_profile_enable(tm_ctx* c, int enable) {
  if (!c) return TM_EINVAL;
  hipSetDevice(c->device);
  prof_drain(c);
  for (int i = 0; i < TM_PROF_MODES; ++i) {
    c->acc_ms[i] = 0;
    c->acc_n[i] = 0;
  }
  c->prof = enable != 0;
  return TM_OK;
}

extern "C" int tm_profile_query(tm_ctx* c, int mode, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return TM_EINVAL;
  if (mode < 0 || mode >= TM_PROF_MODES) return fail(c, TM_EINVAL, "mode %d", mode);
  hipSetDevice(c->device);
  prof_drain(c);
  *ms = c->acc_ms[mode];
  *launches = c->acc_n[mode];
  return TM_OK;
}

// ---------------------------------------------------------------- learned start
static int mlp_check(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, int K, int N, bool train) {
  if (!md || !p) return fail(c, TM_EINVAL, "dims/params pointer is NULL");
  if (md->n_in < 1 || md->hidden < 1 || md->n_out < 1) return fail(c, TM_EINVAL, "network sizes must be positive");
  if (K >= 1 && N >= 1) {
    if (md->n_in != K * N) return fail(c, TM_EINVAL, "n_in=%d must equal K*N=%d", md->n_in, K * N);
    if (md->n_out != 2 * N) return fail(c, TM_EINVAL, "n_out=%d must equal 2N=%d", md->n_out, 2 * N);
  }
  for (int l = 0; l < 3; ++l) {
    if (!p->W[l] || !p->Wh[l] || !p->b[l]) return fail(c, TM_EINVAL, "layer %d weights missing", l);
    if (train && (!p->mW[l] || !p->vW[l] || !p->mb[l] || !p->vb[l]))
      return fail(c, TM_EINVAL, "layer %d Adam moments missing", l);
  }
  return TM_OK;
}

static tmk::MlpParams mlp_params(const tm_mlp_params* p) {
  tmk::MlpParams q;
  for (int l = 0; l < 3; ++l) {
    q.W[l] = p->W[l];
    q.Wh[l] = p->Wh[l];
    q.b[l] = p->b[l];
  }
  return q;
}

static int mlp_run(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, int K, int N, const float* I,
                   int B, tmk::MlpWork& w, void* stream) {
  tmk::MlpShape sh{md->n_in, md->hidden, md->n_out};
  void* base = ws_get(c, WS_PH_BASE + 10, tmk::mlp_work_bytes(sh, B));
  if (!base) return fail(c, TM_ENOMEM, "network workspace");
  tmk::mlp_work_carve(base, sh, B, &w);
  tmk::MlpParams q = mlp_params(p);
  int e = tmk::mlp_forward(sh, q, I, B, K * N, w, stream);
  if (e) return hipfail(c, e, "network forward");
  return TM_OK;
}

extern "C" int tm_mlp_sync_bf16(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, void* stream) {
  if (!c) return TM_EINVAL;
  int r = mlp_check(c, md, p, 0, 0, false);
  if (r) return r;
  HIPCHK(c, hipSetDevice(c->device));
  tmk::MlpShape sh{md->n_in, md->hidden, md->n_out};
  tmk::MlpParams q = mlp_params(p);
  int e = tmk::mlp_weights_to_bf16(sh, q, stream);
  if (e) return hipfail(c, e, "bf16 copy");
  return TM_OK;
}

extern "C" int tm_mlp_start(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, int32_t K, int32_t N,
                            const float* I, int32_t P, tm_c32* t0, void* stream) {
  if (!c) return TM_EINVAL;
  int r = mlp_check(c, md, p, K, N, false);
  if (r) return r;
  if (K < 1 || N < 1 || P < 0) return fail(c, TM_EINVAL, "K, N >= 1 and P >= 0");
  if (P == 0) return TM_OK;
  if (!I || !t0) return fail(c, TM_EINVAL, "null pointer argument");
  HIPCHK(c, hipSetDevice(c->device));
  tmk::MlpWork w;
  if ((r = mlp_run(c, md, p, K, N, I, P, w, stream))) return r;
  int e = tmk::mlp_start(w, P, N, t0, stream);
  if (e) return hipfail(c, e, "network start");
  return TM_OK;
}

static int mlp_grads(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, int K, int N, const float* I,
                     const tm_c32* t, int B, tmk::MlpGrads& G, float* loss, void* stream) {
  tmk::MlpWork w;
  int r = mlp_run(c, md, p, K, N, I, B, w, stream);
  if (r) return r;
  tmk::MlpShape sh{md->n_in, md->hidden, md->n_out};
  tmk::MlpParams q = mlp_params(p);
  int e = tmk::mlp_backward(sh, q, t, B, w, G, stream);
  if (e) return hipfail(c, e, "network backward");
  if (loss) HIPCHK(c, hipMemcpyAsync(loss, w.loss, (size_t)B * sizeof(float), hipMemcpyDeviceToDevice,
                                     (hipStream_t)stream));
  return TM_OK;
}

extern "C" int tm_mlp_gradients(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, int32_t K, int32_t N,
                                const float* I, const tm_c32* t, int32_t B, float* const dW[3],
                                float* const db[3], float* loss, void* stream) {
  if (!c) return TM_EINVAL;
  int r = mlp_check(c, md, p, K, N, false);
  if (r) return r;
  if (B < 1 || !I || !t || !dW || !db) return fail(c, TM_EINVAL, "B >= 1 and non-null arguments");
  for (int l = 0; l < 3; ++l)
    if (!dW[l] || !db[l]) return fail(c, TM_EINVAL, "gradient buffer %d is NULL", l);
  HIPCHK(c, hipSetDevice(c->device));
  tmk::MlpGrads G;
  for (int l = 0; l < 3; ++l) {
    G.dW[l] = dW[l];
    G.db[l] = db[l];
  }
  return mlp_grads(c, md, p, K, N, I, t, B, G, loss, stream);
}

extern "C" int tm_mlp_train_step(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, int32_t K, int32_t N,
                                 const float* I, const tm_c32* t, int32_t B, float lr, int32_t step, float* loss,
                                 void* stream) {
  if (!c) return TM_EINVAL;
  int r = mlp_check(c, md, p, K, N, true);
  if (r) return r;
  if (B < 1 || !I || !t || step < 1 || !(lr >= 0.f)) return fail(c, TM_EINVAL, "B >= 1, step >= 1, lr >= 0");
  HIPCHK(c, hipSetDevice(c->device));
  size_t nw[3] = {(size_t)md->n_in * md->hidden, (size_t)md->hidden * md->hidden, (size_t)md->hidden * md->n_out};
  size_t nb[3] = {(size_t)md->hidden, (size_t)md->hidden, (size_t)md->n_out};
  size_t tot = 0;
  for (int l = 0; l < 3; ++l) tot += ((nw[l] + nb[l]) * 4 + 512);
  char* gb = (char*)ws_get(c, WS_PH_BASE + 11, tot);
  if (!gb) return fail(c, TM_ENOMEM, "gradient workspace");
  tmk::MlpGrads G;
  for (int l = 0; l < 3; ++l) {
    G.dW[l] = (float*)gb;
    gb += (nw[l] * 4 + 255) / 256 * 256;
    G.db[l] = (float*)gb;
    gb += (nb[l] * 4 + 255) / 256 * 256;
  }
  if ((r = mlp_grads(c, md, p, K, N, I, t, B, G, loss, stream))) return r;
  tmk::MlpShape sh{md->n_in, md->hidden, md->n_out};
  tmk::MlpParams q = mlp_params(p);
  tmk::MlpAdam A;
  for (int l = 0; l < 3; ++l) {
    A.mW[l] = p->mW[l];
    A.vW[l] = p->vW[l];
    A.mb[l] = p->mb[l];
    A.vb[l] = p->vb[l];
  }
  int e = tmk::mlp_adam(sh, q, G, A, lr, step, stream);
  if (e) return hipfail(c, e, "Adam");
  return TM_OK;
}

extern "C" int tm_gemm_bf16(tm_ctx* c, int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t ta,
                            const uint16_t* B, int32_t tb, float* C, void* stream) {
  if (!c) return TM_EINVAL;
  if (M < 0 || N < 0 || K < 0) return fail(c, TM_EINVAL, "negative size");
  if (M == 0 || N == 0) return TM_OK;
  if (!A || !B || !C) return fail(c, TM_EINVAL, "null pointer argument");
  HIPCHK(c, hipSetDevice(c->device));
  int e = tmk::gemm_bf16(M, N, K, A, ta != 0, B, tb != 0, C, stream);
  if (e) return hipfail(c, e, "gemm");
  return TM_OK;
}

// ---------------------------------------------------------------- batches
struct tm_batch {
  tm_ctx* c = nullptr;
  std::vector<tm_problem> probs;
  tm_retrieve_opts opts{};
  std::vector<tmk::row_launcher> fns;
  void* dmem = nullptr;
  tmk::BatchArgs args{};
  int grid = 0;
  std::vector<double*> rowsum, sums64;
  std::vector<float*> rowmean, sums;
  std::vector<void*> vprev;
  std::vector<float*> vscale;
  std::vector<void*> lzV;
  std::vector<float*> lzH;
  std::vector<double*> lzY;
  hipStream_t cap = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
};

static int batch_enqueue(tm_batch* b, void* stream) {
  tm_ctx* c = b->c;
  const tm_retrieve_opts& o = b->opts;
  const int n = (int)b->probs.size();
  const int ibf = o.I_dtype == TM_BF16;
  int e = 0;
  if (o.start == TM_START_SPECTRAL) {
    for (int i = 0; i < n; ++i) {
      const tm_problem& p = b->probs[i];
      int N = p.d.n1 * p.d.n2;
      if (p.d.P == 0) continue;
      if (!e) e = tmk::launch_row_isum(p.I, ibf, (int64_t)p.d.K * N, p.d.P, b->rowsum[i], b->rowmean[i], stream);
      if (!e) e = tmk::launch_row_rescale(p.t, N, p.d.P, 0, nullptr, 1.0, stream);
      if (!e) e = tmk::launch_fill_zero(b->vprev[i], (int64_t)p.d.P * N * sizeof(tm_c32), stream);
      if (!e) e = tmk::launch_fill_zero(b->vscale[i], (int64_t)p.d.P * sizeof(float), stream);
    }
    tmk::BatchArgs a = b->args;
    a.tau = o.spectral_tau;
    a.momentum = o.spectral_momentum;
    a.lower = o.spectral_lower;
    for (int it = 0; it < o.spectral_iters && !e; ++it) {
      a.swap = it & 1;  // v and the previous iterate alternate between t and vprev
      e = tmk::batch_launch(tmk::BATCH_SPEC, ibf, 0, a, b->grid, stream);
    }
    for (int i = 0; i < n && !e; ++i) {
      const tm_problem& p = b->probs[i];
      if (!p.d.P) continue;
      const int N = p.d.n1 * p.d.n2;
      if (o.spectral_iters & 1) e = tmk::launch_copy(p.t, b->vprev[i], (int64_t)p.d.P * N * sizeof(tm_c32), stream);
      if (!e) e = tmk::launch_row_rescale(p.t, N, p.d.P, 1, b->rowsum[i], (double)p.d.K * N, stream);
    }
  } else if (o.start == TM_START_LANCZOS) {
    // the first step forms the row sums and means and scales the seeds
    tmk::BatchArgs a = b->args;
    a.tau = o.spectral_tau;
    for (int j = 0; j < o.spectral_iters && !e; ++j) {
      a.lz_j = j;
      e = tmk::batch_launch(tmk::BATCH_LZ, ibf, 0, a, b->grid, stream);
    }
    for (int i = 0; i < n && !e; ++i) {
      const tm_problem& p = b->probs[i];
      if (!p.d.P) continue;
      const int N = p.d.n1 * p.d.n2;
      e = tmk::launch_lz_ritz(b->lzH[i], o.spectral_iters, p.d.P, b->lzY[i], stream);
      if (!e && !ritz_in_sweep(o))
        e = tmk::launch_lz_combine_scaled(p.t, b->lzV[i], b->lzY[i], o.spectral_iters, p.d.P, N, b->rowsum[i],
                                          (double)p.d.K * N, stream);
    }
  } else if (o.start == TM_START_BACKPROP) {
    for (int i = 0; i < n && !e; ++i) {
      const tm_problem& p = b->probs[i];
      tmk::RowArgs a = base_args(c, p.d, p.masks);
      a.I = p.I;
      a.tout = (tmk::cx<float>*)p.t;
      e = b->fns[i](tmk::M_BACKPROP, ibf, a, stream);
    }
  }
  tmk::BatchArgs ea = b->args;
  const bool cyclic = o.method == TM_METHOD_ER_CYCLIC;
  const bool mom = !cyclic && o.er_momentum > 0.f && o.iters > 0;
  if (mom) {
    // t_prev starts equal to t in the per-problem vprev buffer (free after the
    // spectral start); the two buffers then swap roles every iteration
    for (int i = 0; i < n && !e; ++i) {
      const tm_problem& p = b->probs[i];
      if (p.d.P)
        e = tmk::launch_copy(b->vprev[i], p.t, (int64_t)p.d.P * p.d.n1 * p.d.n2 * sizeof(tm_c32), stream);
    }
    ea.er_beta = o.er_momentum;
  }
  for (int it = 0; it < o.iters && !e; ++it) {
    ea.swap = mom ? (it & 1) : 0;
    ea.lz_fuse = (it == 0 && o.start == TM_START_LANCZOS && ritz_in_sweep(o)) ? 1 : 0;
    ea.lz_k = o.spectral_iters;
    e = tmk::batch_launch(cyclic ? tmk::BATCH_ERC : tmk::BATCH_ER, ibf, it == o.iters - 1, ea, b->grid, stream);
  }
  if (mom && (o.iters & 1)) {
    for (int i = 0; i < n && !e; ++i) {
      const tm_problem& p = b->probs[i];
      if (p.d.P)
        e = tmk::launch_copy(p.t, b->vprev[i], (int64_t)p.d.P * p.d.n1 * p.d.n2 * sizeof(tm_c32), stream);
    }
  }
  for (int i = 0; i < n && !e; ++i) {
    const tm_problem& p = b->probs[i];
    if (p.d.P == 0) continue;
    tmk::RowArgs a = base_args(c, p.d, p.masks);
    a.I = p.I;
    a.tin = (const tmk::cx<float>*)p.t;
    a.sums64 = b->sums64[i];
    e = b->fns[i](tmk::M_RES64, ibf, a, stream);
    if (!e && p.stats)
      e = tmk::launch_finalize(p.stats, p.d.P, b->sums64[i], o.iters > 0 ? b->sums[i] : nullptr, tmk::NSUM,
                               o.iters > 0 ? 1 : -1, o.iters > 0 ? 0 : -1, o.iters, 1e-2, stream);
  }
  return e;
}

extern "C" int tm_batch_create(tm_ctx* c, int32_t n, const tm_problem* probs, const tm_retrieve_opts* o,
                               int32_t use_graph, tm_batch** out) {
  if (!c) return TM_EINVAL;
  if (!out || !o || n < 1 || !probs) return fail(c, TM_EINVAL, "n >= 1 and non-null probs, opts, out");
  *out = nullptr;
  if (o->method != TM_METHOD_ER && o->method != TM_METHOD_ER_CYCLIC)
    return fail(c, TM_EUNSUPPORTED, "batches run the error-reduction methods (TM_METHOD_ER, TM_METHOD_ER_CYCLIC)");
  if (!(o->er_momentum >= 0.f && o->er_momentum < 1.f)) return fail(c, TM_EINVAL, "er_momentum must be in [0, 1)");
  if (o->method == TM_METHOD_ER_CYCLIC && o->er_momentum != 0.f)
    return fail(c, TM_EINVAL, "cyclic error reduction takes no momentum (er_momentum must be 0)");
  if (o->iters < 0 || (o->I_dtype != TM_F32 && o->I_dtype != TM_BF16) || o->start < TM_START_GIVEN ||
      o->start > TM_START_LANCZOS)
    return fail(c, TM_EINVAL, "bad options");
  if (o->start == TM_START_LANCZOS && (o->spectral_iters < 1 || o->spectral_iters > tmk::LZ_MAX || !(o->spectral_tau > 0.f)))
    return fail(c, TM_EINVAL, "Lanczos steps (spectral_iters) 1..%d and spectral_tau > 0", tmk::LZ_MAX);
  if (o->start == TM_START_SPECTRAL &&
      (o->spectral_iters < 0 || !(o->spectral_tau > 0.f) || !(o->spectral_momentum >= 0.f && o->spectral_momentum < 1.f) ||
       !(o->spectral_lower >= -1.f && o->spectral_lower <= o->spectral_momentum)))
    return fail(c, TM_EINVAL, "bad spectral options");
  HIPCHK(c, hipSetDevice(c->device));
  tm_batch* b = new tm_batch;
  b->c = c;
  b->opts = *o;
  b->probs.assign(probs, probs + n);
  std::vector<tmk::BatchProb> hp(n);
  std::vector<tmk::BatchItem> items;
  size_t ws_bytes = 0;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const int lzk = o->start == TM_START_LANCZOS ? o->spectral_iters : 0;
  for (int i = 0; i < n; ++i) {
    const tm_problem& p = probs[i];
    tmk::row_launcher fn;
    int r = check_dims(c, p.d, &fn);
    if (r) { delete b; return r; }
    int gid = tmk::batch_grid_id(p.d.n1, p.d.n2);
    if (gid < 0) { delete b; return fail(c, TM_EUNSUPPORTED, "problem %d: grid %dx%d is not compiled for batches", i, p.d.n1, p.d.n2); }
    if (p.d.P > 0 && (!p.masks || !p.I || !p.t)) { delete b; return fail(c, TM_EINVAL, "problem %d: null pointer", i); }
    b->fns.push_back(fn);
    auto v = c->variant.find((ilog2(p.d.n1) << 8) | ilog2(p.d.n2));
    // the batch bodies take the digit order only (eight values per thread in its 512-thread
    // workgroups measured slower: 45.1 against 42.6 ms for 12 problems)
    int var = (v == c->variant.end()) ? 0 : (v->second & 1);
    hp[i].code = 2 * gid + var;
    int rpi = tmk::batch_rows_per_item(gid);
    for (int blk = 0; blk * rpi < p.d.P; ++blk) items.push_back({i, blk});
    size_t N = (size_t)p.d.n1 * p.d.n2;
    ws_bytes += al(p.d.P * 8) + al(p.d.P * 4) + al(p.d.P * tmk::NSUM * 4) + al(p.d.P * 16) + al(p.d.P * N * 8) +
                al(p.d.P * 4);
    if (o->start == TM_START_LANCZOS)
      ws_bytes += al((size_t)lzk * p.d.P * N * 8) + al((size_t)lzk * p.d.P * 8) + al((size_t)lzk * p.d.P * 8);
  }
  size_t tab = al(n * sizeof(tmk::BatchProb)) + al(items.size() * sizeof(tmk::BatchItem));
  if (hipMalloc(&b->dmem, tab + ws_bytes + 256) != hipSuccess) { delete b; return fail(c, TM_ENOMEM, "batch workspace"); }
  char* w = (char*)b->dmem + tab;
  for (int i = 0; i < n; ++i) {
    const tm_problem& p = probs[i];
    size_t N = (size_t)p.d.n1 * p.d.n2;
    b->rowsum.push_back((double*)w); w += al(p.d.P * 8);
    b->rowmean.push_back((float*)w); w += al(p.d.P * 4);
    b->sums.push_back((float*)w); w += al(p.d.P * tmk::NSUM * 4);
    b->sums64.push_back((double*)w); w += al(p.d.P * 16);
    b->vprev.push_back(w); w += al(p.d.P * N * 8);
    b->vscale.push_back((float*)w); w += al(p.d.P * 4);
    b->lzV.push_back(nullptr);
    b->lzH.push_back(nullptr);
    b->lzY.push_back(nullptr);
    if (lzk) {
      b->lzV[i] = w; w += al((size_t)lzk * p.d.P * N * 8);
      b->lzH[i] = (float*)w; w += al((size_t)lzk * p.d.P * 8);
      b->lzY[i] = (double*)w; w += al((size_t)lzk * p.d.P * 8);
    }
    hp[i].lzV = (tmk::cx<float>*)b->lzV[i];
    hp[i].lzH = b->lzH[i];
    hp[i].lzY = b->lzY[i];
    hp[i].N = (int)N;
    hp[i].masks = (const tmk::cx<float>*)p.masks;
    hp[i].I = p.I;
    hp[i].t = (tmk::cx<float>*)p.t;
    hp[i].vprev = (tmk::cx<float>*)b->vprev[i];
    hp[i].vscale = b->vscale[i];
    hp[i].sums = b->sums[i];
    hp[i].rowmean = b->rowmean[i];
    hp[i].rowsum = b->rowsum[i];
    hp[i].K = p.d.K;
    hp[i].P = p.d.P;
  }
  tmk::BatchProb* dprobs = (tmk::BatchProb*)b->dmem;
  tmk::BatchItem* ditems = (tmk::BatchItem*)((char*)b->dmem + al(n * sizeof(tmk::BatchProb)));
  if (hipMemcpy(dprobs, hp.data(), n * sizeof(tmk::BatchProb), hipMemcpyHostToDevice) != hipSuccess ||
      (!items.empty() && hipMemcpy(ditems, items.data(), items.size() * sizeof(tmk::BatchItem), hipMemcpyHostToDevice) != hipSuccess)) {
    hipFree(b->dmem);
    delete b;
    return fail(c, TM_EHIP, "batch table upload");
  }
  b->args.probs = dprobs;
  b->args.items = ditems;
  b->args.n_items = (int)items.size();
  b->args.tw32 = c->tw32;
  // persistent grid: every CU holds one 512-thread workgroup (LDS and registers)
  int cus = 0;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
  b->grid = std::max(1, std::min((int)items.size(), cus > 0 ? cus : 256));
  if (use_graph) {
    hipError_t he = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
    int e = (he == hipSuccess) ? batch_enqueue(b, b->cap) : (int)he;
    hipGraph_t g = nullptr;
    hipError_t he2 = b->cap ? hipStreamEndCapture(b->cap, &g) : hipErrorInvalidValue;
    if (!e && he2 == hipSuccess) {
      b->g = g;
      he2 = hipGraphInstantiate(&b->ge, g, nullptr, nullptr, 0);
    }
    if (e || he2 != hipSuccess) {
      int code = e ? e : (int)he2;
      tm_batch_destroy(b);
      return hipfail(c, code, "batch graph capture");
    }
  }
  *out = b;
  return TM_OK;
}

extern "C" int tm_batch_run(tm_batch* b, void* stream) {
  if (!b) return TM_EINVAL;
  tm_ctx* c = b->c;
  HIPCHK(c, hipSetDevice(c->device));
  if (b->ge) {
    HIPCHK(c, hipGraphLaunch(b->ge, (hipStream_t)stream));
    return TM_OK;
  }
  int e = batch_enqueue(b, stream);
  if (e) return hipfail(c, e, "batch launch");
  return TM_OK;
}

extern "C" int tm_batch_destroy(tm_batch* b) {
  if (!b) return TM_EINVAL;
  hipSetDevice(b->c->device);
  hipDeviceSynchronize();
  if (b->ge) hipGraphExecDestroy(b->ge);
  if (b->g) hipGraphDestroy(b->g);
  if (b->cap) hipStreamDestroy(b->cap);
  hipFree(b->dmem);
  delete b;
  return TM_OK;
}

// ---------------------------------------------------------------- autotuning
extern "C" int tm_set_variant(tm_ctx* c, int32_t n1, int32_t n2, int32_t variant) {
  if (!c) return TM_EINVAL;
  if (variant < 0 || variant > 1) return fail(c, TM_EINVAL, "variant %d", variant);
  if (!tm_grid_supported(n1, n2)) return fail(c, TM_EUNSUPPORTED, "grid %dx%d", n1, n2);
  c->variant[(ilog2(n1) << 8) | ilog2(n2)] = variant;
  return TM_OK;
}

extern "C" int tm_tune_time(tm_ctx* c, int32_t n1, int32_t n2, int32_t K, int32_t P, int32_t I_dtype,
                            int32_t variant, int32_t reps, double* us) {
  if (!c) return TM_EINVAL;
  if (!us || reps < 1 || P < 1 || K < 1 || variant < 0 || variant > 1 || (I_dtype != TM_F32 && I_dtype != TM_BF16))
    return fail(c, TM_EINVAL, "bad tuning arguments");
  tm_dims d{n1, n2, K, P};
  tmk::row_launcher fn0;
  int r = check_dims(c, d, &fn0);
  if (r) return r;
  tmk::row_launcher fn = tmk::find_row_launcher(ilog2(n1), ilog2(n2), variant);
  HIPCHK(c, hipSetDevice(c->device));
  size_t N = (size_t)n1 * n2;
  float* mk = (float*)ws_get(c, WS_PH_BASE + 20, K * N * 8);
  float* t = (float*)ws_get(c, WS_PH_BASE + 21, P * N * 8);
  float* I = (float*)ws_get(c, WS_PH_BASE + 22, (size_t)P * K * N * 4);
  if (!mk || !t || !I) return fail(c, TM_ENOMEM, "tuning workspace");
  hipStream_t s = nullptr;
  int e = tmk::launch_fill_hash(mk, (int64_t)K * N * 2, 11u, -0.7f, 0.7f, s);
  if (!e) e = tmk::launch_fill_hash(t, (int64_t)P * N * 2, 12u, -1.f, 1.f, s);
  // intensities in [0.5, 2); read as bf16 the buffer holds arbitrary values,
  // which leaves the timing unchanged (only the timing is used)
  if (!e) e = tmk::launch_fill_hash(I, (int64_t)P * K * N, 13u, 0.5f, 2.f, s);
  if (e) return hipfail(c, e, "tuning data");
  tmk::RowArgs a = base_args(c, d, (const tm_c32*)mk);
  a.I = I;
  a.tin = (const tmk::cx<float>*)t;
  a.tout = (tmk::cx<float>*)t;
  int ibf = I_dtype == TM_BF16;
  if ((e = fn(tmk::M_ER, ibf, a, s))) return hipfail(c, e, "tuning warm-up");
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  hipEventRecord(e0, s);
  for (int i = 0; i < reps && !e; ++i) e = fn(tmk::M_ER, ibf, a, s);
  hipEventRecord(e1, s);
  hipEventSynchronize(e1);
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e) return hipfail(c, e, "tuning launch");
  *us = 1e3 * ms / reps;
  return TM_OK;
}

extern "C" int tm_config_info(int32_t n1, int32_t n2, int32_t cfg, int32_t* wg, int32_t* rows_per_wg,
                              int32_t* values_per_thread) {
  if (!is_pow2(n1) || !is_pow2(n2) || (int64_t)n1 * n2 > TW_MAX || cfg < 0 || cfg > 7) return 0;
  const int L1 = ilog2(n1), L2 = ilog2(n2);
  if (!((tmk::row_cfg_mask(L1, L2) >> cfg) & 1)) return 0;
  int w = 0, r = 0, e = 0;
  tmk::row_cfg_shape(L1, L2, cfg, &w, &r, &e);
  if (wg) *wg = w;
  if (rows_per_wg) *rows_per_wg = r;
  if (values_per_thread) *values_per_thread = e;
  return 1;
}

extern "C" int tm_set_config(tm_ctx* c, int32_t n1, int32_t n2, int32_t cfg) {
  if (!c) return TM_EINVAL;
  if (!tm_grid_supported(n1, n2)) return fail(c, TM_EUNSUPPORTED, "grid %dx%d", n1, n2);
  if (!tm_config_info(n1, n2, cfg, nullptr, nullptr, nullptr))
    return fail(c, TM_EUNSUPPORTED, "configuration %d is not compiled for grid %dx%d", cfg, n1, n2);
  c->variant[(ilog2(n1) << 8) | ilog2(n2)] = cfg;
  return TM_OK;
}

extern "C" int tm_tune_config(tm_ctx* c, int32_t n1, int32_t n2, int32_t K, int32_t P, int32_t I_dtype, int32_t cfg,
                              int32_t reps, double* us) {
  if (!c) return TM_EINVAL;
  if (!us || reps < 1 || P < 1 || K < 1 || (I_dtype != TM_F32 && I_dtype != TM_BF16))
    return fail(c, TM_EINVAL, "bad tuning arguments");
  tm_dims d{n1, n2, K, P};
  tmk::row_launcher fn0;
  int r = check_dims(c, d, &fn0);
  if (r) return r;
  if (!tm_config_info(n1, n2, cfg, nullptr, nullptr, nullptr))
    return fail(c, TM_EUNSUPPORTED, "configuration %d is not compiled for grid %dx%d", cfg, n1, n2);
  tmk::row_launcher fn = tmk::find_row_launcher(ilog2(n1), ilog2(n2), cfg);
  HIPCHK(c, hipSetDevice(c->device));
  size_t N = (size_t)n1 * n2;
  float* mk = (float*)ws_get(c, WS_PH_BASE + 20, K * N * 8);
  float* t = (float*)ws_get(c, WS_PH_BASE + 21, P * N * 8);
  float* I = (float*)ws_get(c, WS_PH_BASE + 22, (size_t)P * K * N * 4);
  float* t2 = (float*)ws_get(c, WS_PH_BASE + 23, P * N * 8);
  float* rm = (float*)ws_get(c, WS_PH_BASE + 24, (size_t)P * 4);
  float* lz = (float*)ws_get(c, WS_PH_BASE + 25, (size_t)P * 8);
  if (!mk || !t || !I || !t2 || !rm || !lz) return fail(c, TM_ENOMEM, "tuning workspace");
  hipStream_t s = nullptr;
  int e = tmk::launch_fill_hash(mk, (int64_t)K * N * 2, 11u, -0.7f, 0.7f, s);
  if (!e) e = tmk::launch_fill_hash(t, (int64_t)P * N * 2, 12u, -1.f, 1.f, s);
  if (!e) e = tmk::launch_fill_hash(I, (int64_t)P * K * N, 13u, 0.5f, 2.f, s);  // see tm_tune_time
  if (!e) e = tmk::launch_fill_hash(rm, (int64_t)P, 14u, 1.f, 1.f, s);
  if (e) return hipfail(c, e, "tuning data");
  const int ibf = I_dtype == TM_BF16;
  tmk::RowArgs lz_a = base_args(c, d, (const tm_c32*)mk);
  lz_a.I = I;
  lz_a.tin = lz_a.din = (const tmk::cx<float>*)t;
  lz_a.tout = (tmk::cx<float>*)t2;
  lz_a.rowmean = rm;
  lz_a.tau = 3.f;
  lz_a.lz_out = lz;
  tmk::RowArgs er_a = base_args(c, d, (const tm_c32*)mk);
  er_a.I = I;
  er_a.tin = (const tmk::cx<float>*)t2;
  er_a.tout = (tmk::cx<float>*)t2;
  const int modes[2] = {tmk::M_LANCZOS, tmk::M_ERC};
  const tmk::RowArgs* args[2] = {&lz_a, &er_a};
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  for (int k = 0; k < 2 && !e; ++k) {
    e = fn(modes[k], ibf, *args[k], s);  // warm-up
    hipEventRecord(e0, s);
    for (int i = 0; i < reps && !e; ++i) e = fn(modes[k], ibf, *args[k], s);
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    us[k] = 1e3 * ms / reps;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e) return hipfail(c, e, "tuning launch");
  return TM_OK;
}

// ------------------------------------------------------------ preprocessing
static int pre_check(tm_ctx* c, const void* stack, int32_t dtype, int64_t n_img, int32_t H, int32_t W) {
  if (!stack) return fail(c, TM_EINVAL, "stack is NULL");
  if (dtype != TM_F32 && dtype != TM_U16) return fail(c, TM_EINVAL, "stack dtype %d (TM_F32 or TM_U16)", dtype);
  if (n_img < 1) return fail(c, TM_EINVAL, "n_img=%lld must be >= 1", (long long)n_img);
  if (H < 2 || W < 2 || (H & 1) || (W & 1)) return fail(c, TM_EINVAL, "image %dx%d: even sizes >= 2", H, W);
  if ((int64_t)(H / 2) * (W / 2) > (int64_t)1 << 30) return fail(c, TM_EINVAL, "image too large");
  return TM_OK;
}

extern "C" int tm_pre_energy(tm_ctx* c, const void* stack, int32_t stack_dtype, int64_t n_img, int32_t H, int32_t W,
                             double* energy, void* stream) {
  if (!c) return TM_EINVAL;
  int r = pre_check(c, stack, stack_dtype, n_img, H, W);
  if (r) return r;
  if (!energy) return fail(c, TM_EINVAL, "energy is NULL");
  HIPCHK(c, hipSetDevice(c->device));
  const int npix = (H / 2) * (W / 2);
  const int nch = tmk::pre_energy_chunks(stack, stack_dtype == TM_U16, n_img, H, W);
  double* part = (double*)ws_get(c, WS_PRE_PART, (size_t)nch * npix * sizeof(double));
  if (!part) return fail(c, TM_ENOMEM, "workspace");
  int e = tmk::launch_pre_energy(stack, stack_dtype == TM_U16, n_img, H, W, part, nch, energy, stream);
  if (e) return hipfail(c, e, "energy");
  return TM_OK;
}

extern "C" int tm_pre_fiber_mask(tm_ctx* c, const double* energy, int32_t npix, double frac, int32_t* pix,
                                 int32_t* P_out, void* stream) {
  if (!c) return TM_EINVAL;
  if (!energy || !pix || !P_out) return fail(c, TM_EINVAL, "null pointer argument");
  if (npix < 1 || npix > tmk::PRE_MASK_MAX) return fail(c, TM_EINVAL, "npix=%d outside 1..%d", npix, tmk::PRE_MASK_MAX);
  if (!(frac > 0.0 && frac <= 1.0)) return fail(c, TM_EINVAL, "frac must be in (0, 1]");
  HIPCHK(c, hipSetDevice(c->device));
  int32_t* cnt = (int32_t*)ws_get(c, WS_PRE_COUNT, sizeof(int32_t));
  if (!cnt) return fail(c, TM_ENOMEM, "workspace");
  int e = tmk::launch_pre_mask(energy, npix, frac, pix, cnt, stream);
  if (e) return hipfail(c, e, "fiber mask");
  int32_t h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
  *P_out = h;
  return TM_OK;
}

extern "C" int tm_pre_gather(tm_ctx* c, const void* stack, int32_t stack_dtype, int64_t n_img, int32_t H, int32_t W,
                             const int32_t* pix, int32_t P, void* out, int32_t out_dtype, void* stream) {
  if (!c) return TM_EINVAL;
  int r = pre_check(c, stack, stack_dtype, n_img, H, W);
  if (r) return r;
  if (P < 0) return fail(c, TM_EINVAL, "P=%d < 0", P);
  if (out_dtype != TM_F32 && out_dtype != TM_BF16) return fail(c, TM_EINVAL, "out dtype %d (TM_F32 or TM_BF16)", out_dtype);
  if (P == 0) return TM_OK;
  if (!pix || !out) return fail(c, TM_EINVAL, "null pointer argument");
  HIPCHK(c, hipSetDevice(c->device));
  // the pixel indices address the half-sampled grid: check them on the host
  const int npix = (H / 2) * (W / 2);
  std::vector<int32_t> hp(P);
  if (hipMemcpy(hp.data(), pix, (size_t)P * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, TM_EHIP, "reading pix");
  for (int i = 0; i < P; ++i)
    if (hp[i] < 0 || hp[i] >= npix) return fail(c, TM_EINVAL, "pix[%d]=%d outside the half-sampled grid", i, hp[i]);
  int e = tmk::launch_pre_gather(stack, stack_dtype == TM_U16, n_img, H, W, pix, P, out, out_dtype == TM_BF16, stream);
  if (e) return hipfail(c, e, "gather");
  return TM_OK;
}

// ------------------------------------------------------------ foci and power ratio

extern "C" int tm_foci_power_ratio(tm_ctx* c, int32_t Pf, int32_t G, int32_t N, const tm_c32* tm_true,
                                   const int32_t* pix, const tm_c32* tm_est, int32_t g1, int32_t g2, int32_t w,
                                   float* pr, int32_t* peak, void* stream) {
  if (!c) return TM_EINVAL;
  if (Pf < 0 || G < 1 || N < 1 || g1 < 1 || g2 < 1 || w < 0)
    return fail(c, TM_EINVAL, "Pf >= 0, G >= 1, N >= 1, grid >= 1, w >= 0");
  if (Pf == 0) return TM_OK;
  if (!tm_true || !tm_est || !pix || !pr || !peak) return fail(c, TM_EINVAL, "null pointer argument");
  if ((int64_t)G > (int64_t)g1 * g2) return fail(c, TM_EINVAL, "G=%d exceeds the %dx%d grid", G, g1, g2);
  HIPCHK(c, hipSetDevice(c->device));
  std::vector<int32_t> hp(G);
  if (hipMemcpy(hp.data(), pix, (size_t)G * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, TM_EHIP, "reading pix");
  std::vector<char> seen((size_t)g1 * g2, 0);
  for (int i = 0; i < G; ++i) {
    if (hp[i] < 0 || hp[i] >= g1 * g2) return fail(c, TM_EINVAL, "pix[%d]=%d outside the grid", i, hp[i]);
    if (seen[hp[i]]) return fail(c, TM_EINVAL, "pix[%d]=%d repeats a pixel", i, hp[i]);
    seen[hp[i]] = 1;
  }
  void* u = ws_get(c, WS_FOCI_U, (size_t)Pf * N * sizeof(tm_c32));
  void* E = ws_get(c, WS_FOCI_E, (size_t)Pf * G * sizeof(tm_c32));
  if (!u || !E) return fail(c, TM_ENOMEM, "workspace");
  int e = tmk::launch_conj_phase(tm_est, u, (int64_t)Pf * N, stream);
  if (e) return hipfail(c, e, "conjugate phase");
  // E[p][q] = sum_n u[p][n] tm_true[q][n] (both operands n-contiguous)
  e = tmk::launch_cgemm(Pf, G, N, u, N, tm_true, N, 1, E, G, 0, stream);
  if (e) return hipfail(c, e, "foci GEMM");
  e = tmk::launch_foci_pr(E, Pf, G, pix, g1, g2, w, pr, peak, stream);
  if (e) return hipfail(c, e, "power ratio");
  return TM_OK;
}

// ------------------------------------------------------------ dense-probing comparator
extern "C" int tm_cgemm_f32(tm_ctx* c, int32_t M, int32_t N, int32_t K, const tm_c32* A, int64_t lda,
                            const tm_c32* B, int64_t ldb, int32_t trans_b, tm_c32* C, int64_t ldc, int32_t conj_c,
                            void* stream) {
  if (!c) return TM_EINVAL;
  if (M < 0 || N < 0 || K < 1) return fail(c, TM_EINVAL, "M, N >= 0 and K >= 1");
  if (M == 0 || N == 0) return TM_OK;
  if (!A || !B || !C) return fail(c, TM_EINVAL, "null pointer argument");
  if (lda < K || (trans_b ? ldb < K : ldb < N) || ldc < N) return fail(c, TM_EINVAL, "leading dimensions too small");
  if ((M + 127) / 128 > 65535) return fail(c, TM_EINVAL, "M=%d too large", M);
  HIPCHK(c, hipSetDevice(c->device));
  int e = tmk::launch_cgemm(M, N, K, A, lda, B, ldb, trans_b ? 1 : 0, C, ldc, conj_c ? 1 : 0, stream);
  if (e) return hipfail(c, e, "complex GEMM");
  return TM_OK;
}

extern "C" int tm_dense_gradient(tm_ctx* c, int32_t M, int32_t N, int32_t P, const tm_c32* Q, const float* I,
                                 const tm_c32* t, tm_c32* grad, float* f, void* stream) {
  if (!c) return TM_EINVAL;
  if (M < 1 || N < 1 || P < 0) return fail(c, TM_EINVAL, "M, N >= 1 and P >= 0");
  if (P == 0) return TM_OK;
  if (!Q || !I || !t || !grad) return fail(c, TM_EINVAL, "null pointer argument");
  HIPCHK(c, hipSetDevice(c->device));
  void* Y = ws_get(c, WS_DENSE_Y, (size_t)P * M * sizeof(tm_c32));
  if (!Y) return fail(c, TM_ENOMEM, "workspace");
  // Y [P][M] = t Q^T (both operands n-contiguous)
  int e = tmk::launch_cgemm(P, M, N, t, N, Q, N, 1, Y, M, 0, stream);
  if (e) return hipfail(c, e, "dense GEMM");
  e = tmk::launch_dense_pointwise(Y, I, P, M, f, stream);
  if (e) return hipfail(c, e, "dense pointwise");
  // grad [P][N] = conj(Y' Q) with Y' = conj(w) from the pointwise kernel (Q read [M][N], n-contiguous)
  e = tmk::launch_cgemm(P, N, M, Y, M, Q, N, 0, grad, N, 1, stream);
  if (e) return hipfail(c, e, "dense GEMM");
  return TM_OK;
}

// ------------------------------------------------------------ propagated TM
extern "C" int tm_propagate_tm(tm_ctx* c, int32_t P, int32_t N, const tm_c32* tm, const int32_t* pix, int32_t g1,
                               int32_t g2, const tm_optics* o, tm_c32* out, void* stream) {
  if (!c) return TM_EINVAL;
  if (P < 0 || N < 1) return fail(c, TM_EINVAL, "P >= 0 and N >= 1");
  if (!o || !out || (P > 0 && (!tm || !pix))) return fail(c, TM_EINVAL, "null pointer argument");
  if (!(o->lambda > 0) || !(o->ps_field > 0) || !(o->NA > 0) || !std::isfinite(o->z))
    return fail(c, TM_EINVAL, "optics: lambda, ps_field, NA > 0 and finite z");
  tmk::row_launcher fn;
  tm_dims gd{g1, g2, 1, N};  // the grid's 2-D FFT is the row kernel's, one "row" per TM column
  int r = check_dims(c, gd, &fn);
  if (r) return r;
  const int G = g1 * g2;
  if (P > G) return fail(c, TM_EINVAL, "P=%d exceeds the %dx%d grid", P, g1, g2);
  HIPCHK(c, hipSetDevice(c->device));
  if (P > 0) {
    std::vector<int32_t> hp(P);
    if (hipMemcpy(hp.data(), pix, (size_t)P * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(c, TM_EHIP, "reading pix");
    std::vector<char> seen((size_t)G, 0);
    for (int i = 0; i < P; ++i) {
      if (hp[i] < 0 || hp[i] >= G) return fail(c, TM_EINVAL, "pix[%d]=%d outside the grid", i, hp[i]);
      if (seen[hp[i]]) return fail(c, TM_EINVAL, "pix[%d]=%d repeats a pixel", i, hp[i]);
      seen[hp[i]] = 1;
    }
  }
  void* X = ws_get(c, WS_PROP_X, (size_t)N * G * sizeof(tm_c32));
  void* H = ws_get(c, WS_PROP_H, (size_t)G * sizeof(tm_c32));
  void* ones = ws_get(c, WS_PROP_ONES, (size_t)G * sizeof(tm_c32));
  if (!X || !H || !ones) return fail(c, TM_ENOMEM, "workspace");
  int e = tmk::launch_fill_c32(X, (int64_t)N * G, 0.f, 0.f, stream);
  if (!e) e = tmk::launch_fill_c32(ones, G, 1.f, 0.f, stream);
  if (!e) e = tmk::launch_cols_to_grid(tm, P, N, pix, G, X, stream);
  if (!e) e = tmk::launch_make_prop_filter(H, g1, g2, o->lambda, o->ps_field, o->NA, o->z, stream);
  if (e) return hipfail(c, e, "propagation setup");
  tmk::RowArgs a = base_args(c, gd, (const tm_c32*)ones);
  a.tin = (const tmk::cx<float>*)X;
  a.tout = (tmk::cx<float>*)X;
  a.yin = (const tmk::cx<float>*)H;
  r = run_row(c, fn, tmk::M_FILT, 0, a, stream);
  if (r) return r;
  e = tmk::launch_grid_to_rows(X, N, G, out, stream);
  if (e) return hipfail(c, e, "transpose");
  return TM_OK;
}

// ---------------------------------------------------------------- learned weights of the spectral start
static int wnet_check(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, int nt, float xmax, bool train) {
  if (!md || !p) return fail(c, TM_EINVAL, "dims/params pointer is NULL");
  if (md->n_in != tmk::WNET_FEATURES || md->n_out != 1 || md->hidden < 1 || md->hidden > 4096)
    return fail(c, TM_EINVAL, "weight network must be %d -> hidden (1..4096) -> hidden -> 1", tmk::WNET_FEATURES);
  if (nt < 2 || nt > TM_WTAB_MAX) return fail(c, TM_EINVAL, "table points %d outside 2..%d", nt, TM_WTAB_MAX);
  if (!(xmax > 0.f) || !std::isfinite(xmax)) return fail(c, TM_EINVAL, "xmax must be > 0");
  return mlp_check(c, md, p, 0, 0, train);
}

// network forward on the table points; outputs in w.O [nt]
static int wnet_forward(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, int nt, float xmax,
                        tmk::MlpWork& w, void* stream) {
  tmk::MlpShape sh{md->n_in, md->hidden, md->n_out};
  void* base = ws_get(c, WS_PH_BASE + 30, tmk::mlp_work_bytes(sh, nt));
  if (!base) return fail(c, TM_ENOMEM, "network workspace");
  tmk::mlp_work_carve(base, sh, nt, &w);
  int e = tmk::wnet_features(nt, xmax, w.X, stream);
  tmk::MlpParams q = mlp_params(p);
  if (!e) e = tmk::mlp_forward_x(sh, q, nt, w, stream);
  if (e) return hipfail(c, e, "weight network forward");
  return TM_OK;
}

// backward from w.dOh / w.dOf, Adam on the masters and the BF16 copies refreshed
static int wnet_update(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, int nt, tmk::MlpWork& w, float lr,
                       int step, void* stream) {
  size_t nw[3] = {(size_t)md->n_in * md->hidden, (size_t)md->hidden * md->hidden, (size_t)md->hidden * md->n_out};
  size_t nb[3] = {(size_t)md->hidden, (size_t)md->hidden, (size_t)md->n_out};
  size_t tot = 0;
  for (int l = 0; l < 3; ++l) tot += ((nw[l] + nb[l]) * 4 + 512);
  char* gb = (char*)ws_get(c, WS_PH_BASE + 31, tot);
  if (!gb) return fail(c, TM_ENOMEM, "gradient workspace");
  tmk::MlpGrads G;
  for (int l = 0; l < 3; ++l) {
    G.dW[l] = (float*)gb;
    gb += (nw[l] * 4 + 255) / 256 * 256;
    G.db[l] = (float*)gb;
    gb += (nb[l] * 4 + 255) / 256 * 256;
  }
  tmk::MlpShape sh{md->n_in, md->hidden, md->n_out};
  tmk::MlpParams q = mlp_params(p);
  int e = tmk::mlp_backward_dout(sh, q, nt, w, G, stream);
  if (e) return hipfail(c, e, "weight network backward");
  tmk::MlpAdam A;
  for (int l = 0; l < 3; ++l) {
    A.mW[l] = p->mW[l];
    A.vW[l] = p->vW[l];
    A.mb[l] = p->mb[l];
    A.vb[l] = p->vb[l];
  }
  e = tmk::mlp_adam(sh, q, G, A, lr, step, stream);
  if (e) return hipfail(c, e, "Adam");
  return TM_OK;
}

extern "C" int tm_wnet_table(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, int32_t nt, float xmax,
                             float* tab, void* stream) {
  if (!c) return TM_EINVAL;
  int r = wnet_check(c, md, p, nt, xmax, false);
  if (r) return r;
  if (!tab) return fail(c, TM_EINVAL, "tab is NULL");
  HIPCHK(c, hipSetDevice(c->device));
  tmk::MlpWork w;
  if ((r = wnet_forward(c, md, p, nt, xmax, w, stream))) return r;
  int e = tmk::wnet_pairs(w.O, nt, tab, stream);
  if (e) return hipfail(c, e, "table");
  return TM_OK;
}

extern "C" int tm_wnet_pretrain_step(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, int32_t nt,
                                     float xmax, float tau, float lr, int32_t step, float* loss, void* stream) {
  if (!c) return TM_EINVAL;
  int r = wnet_check(c, md, p, nt, xmax, true);
  if (r) return r;
  if (step < 1 || !(lr >= 0.f) || !(tau > 0.f)) return fail(c, TM_EINVAL, "step >= 1, lr >= 0, tau > 0");
  HIPCHK(c, hipSetDevice(c->device));
  tmk::MlpWork w;
  if ((r = wnet_forward(c, md, p, nt, xmax, w, stream))) return r;
  int e = tmk::wnet_regress(w.O, nt, xmax, tau, w.dOf, w.dOh, loss ? loss : w.loss, stream);
  if (e) return hipfail(c, e, "regression");
  return wnet_update(c, md, p, nt, w, lr, step, stream);
}

// Loss of k normalised power steps with the table's weights and its gradient
// with respect to the table (dtab, overwritten).
static int wtab_grad(tm_ctx* c, tmk::row_launcher fn, const tm_dims& d, const tm_c32* masks, const void* I, int ibf,
                     const tm_c32* t, const tm_c32* v0, int k, const float* tab, int nt, float xmax, float* dtab,
                     float* loss, void* stream) {
  const int N = d.n1 * d.n2, B = d.P;
  const size_t row = (size_t)B * N * sizeof(tm_c32);
  char* U = (char*)ws_get(c, WS_PH_BASE + 32, row * (k + 1));
  void* Y = ws_get(c, WS_PH_BASE + 33, row);
  void* G = ws_get(c, WS_PH_BASE + 34, row);
  void* Gy = ws_get(c, WS_PH_BASE + 35, row);
  float* gw = (float*)ws_get(c, WS_PH_BASE + 36, (size_t)B * d.K * N * sizeof(float));
  float* nrm = (float*)ws_get(c, WS_PH_BASE + 37, (size_t)k * B * sizeof(float));
  float* fid = (float*)ws_get(c, WS_PH_BASE + 38, (size_t)B * sizeof(float));
  double* rowsum = (double*)ws_get(c, WS_ROWSUM, (size_t)B * sizeof(double));
  float* rowmean = (float*)ws_get(c, WS_ROWMEAN, (size_t)B * sizeof(float));
  float* sums = (float*)ws_get(c, WS_SUMS, (size_t)B * tmk::NSUM * sizeof(float));
  if (!U || !Y || !G || !Gy || !gw || !nrm || !fid || !rowsum || !rowmean || !sums)
    return fail(c, TM_ENOMEM, "training workspace");
  auto Uj = [&](int j) { return (void*)(U + row * j); };
  int e = tmk::launch_row_isum(I, ibf, (int64_t)d.K * N, B, rowsum, rowmean, stream);
  if (!e) e = tmk::launch_copy(Uj(0), v0, (int64_t)row, stream);
  if (!e) e = tmk::launch_row_rescale(Uj(0), N, B, 0, nullptr, 1.0, stream);
  if (!e) e = tmk::launch_fill_zero(dtab, (int64_t)nt * sizeof(float), stream);
  if (e) return hipfail(c, e, "training setup");
  tmk::RowArgs a = base_args(c, d, masks);
  a.I = I;
  a.rowmean = rowmean;
  a.wtab = tab;
  a.wtab_scale = (float)(nt - 1) / xmax;
  a.wtab_last = (float)(nt - 1);
  a.sums = sums;
  int r;
  for (int j = 0; j < k; ++j) {
    a.tin = (const tmk::cx<float>*)Uj(j);
    a.tout = (tmk::cx<float>*)Y;
    if ((r = run_row(c, fn, tmk::M_WAPPLY, ibf, a, stream))) return r;
    e = tmk::wnet_normalise(Y, sums, tmk::NSUM, B, N, Uj(j + 1), nrm + (size_t)j * B, stream);
    if (e) return hipfail(c, e, "normalise");
  }
  e = tmk::wnet_loss(Uj(k), t, B, N, G, fid, loss, stream);
  if (e) return hipfail(c, e, "loss");
  for (int j = k - 1; j >= 0; --j) {
    e = tmk::wnet_normback(G, Uj(j + 1), nrm + (size_t)j * B, B, N, Gy, stream);
    if (e) return hipfail(c, e, "normalisation backward");
    a.tin = (const tmk::cx<float>*)Uj(j);
    a.din = (const tmk::cx<float>*)Gy;
    a.yout = gw;
    a.tout = (tmk::cx<float>*)G;
    if ((r = run_row(c, fn, tmk::M_WBACK, ibf, a, stream))) return r;
    e = tmk::wnet_hist(gw, I, ibf, rowmean, B, d.K * N, nt, xmax, dtab, stream);
    if (e) return hipfail(c, e, "table gradient");
  }
  return TM_OK;
}

static int wtab_args(tm_ctx* c, const tm_dims& d, tmk::row_launcher* fn, const tm_c32* masks, const void* I,
                     int I_dtype, const tm_c32* t, const tm_c32* v0, int k, int nt, float xmax) {
  int r = check_dims(c, d, fn);
  if (r) return r;
  if (d.P < 1) return fail(c, TM_EINVAL, "P >= 1 training rows");
  if (k < 1 || k > 256) return fail(c, TM_EINVAL, "power steps %d outside 1..256", k);
  if (nt < 2 || nt > TM_WTAB_MAX) return fail(c, TM_EINVAL, "table points %d outside 2..%d", nt, TM_WTAB_MAX);
  if (!(xmax > 0.f) || !std::isfinite(xmax)) return fail(c, TM_EINVAL, "xmax must be > 0");
  if (I_dtype != TM_F32 && I_dtype != TM_BF16) return fail(c, TM_EINVAL, "I_dtype %d", I_dtype);
  if (!masks || !I || !t || !v0) return fail(c, TM_EINVAL, "null pointer argument");
  return TM_OK;
}

extern "C" int tm_wtab_power_grad(tm_ctx* c, tm_dims d, const tm_c32* masks, const void* I, int32_t I_dtype,
                                  const tm_c32* t, const tm_c32* v0, int32_t steps, const float* tab, int32_t nt,
                                  float xmax, float* dtab, float* loss, void* stream) {
  if (!c) return TM_EINVAL;
  tmk::row_launcher fn;
  int r = wtab_args(c, d, &fn, masks, I, I_dtype, t, v0, steps, nt, xmax);
  if (r) return r;
  if (!tab || !dtab || !loss) return fail(c, TM_EINVAL, "null pointer argument");
  HIPCHK(c, hipSetDevice(c->device));
  return wtab_grad(c, fn, d, masks, I, I_dtype == TM_BF16, t, v0, steps, tab, nt, xmax, dtab, loss, stream);
}

extern "C" int tm_wnet_train_step(tm_ctx* c, const tm_mlp_dims* md, const tm_mlp_params* p, tm_dims d,
                                  const tm_c32* masks, const void* I, int32_t I_dtype, const tm_c32* t,
                                  const tm_c32* v0, int32_t steps, int32_t nt, float xmax, float lr, int32_t step,
                                  float* loss, void* stream) {
  if (!c) return TM_EINVAL;
  int r = wnet_check(c, md, p, nt, xmax, true);
  if (r) return r;
  tmk::row_launcher fn;
  if ((r = wtab_args(c, d, &fn, masks, I, I_dtype, t, v0, steps, nt, xmax))) return r;
  if (step < 1 || !(lr >= 0.f)) return fail(c, TM_EINVAL, "step >= 1, lr >= 0");
  HIPCHK(c, hipSetDevice(c->device));
  tmk::MlpWork w;
  if ((r = wnet_forward(c, md, p, nt, xmax, w, stream))) return r;
  float* tab = (float*)ws_get(c, WS_PH_BASE + 39, (size_t)nt * 2 * sizeof(float));
  float* dtab = (float*)ws_get(c, WS_PH_BASE + 40, (size_t)nt * sizeof(float));
  if (!tab || !dtab) return fail(c, TM_ENOMEM, "table workspace");
  int e = tmk::wnet_pairs(w.O, nt, tab, stream);
  if (e) return hipfail(c, e, "table");
  if ((r = wtab_grad(c, fn, d, masks, I, I_dtype == TM_BF16, t, v0, steps, tab, nt, xmax, dtab,
                     loss ? loss : w.loss, stream)))
    return r;
  e = tmk::wnet_dout(dtab, nt, w.dOf, w.dOh, stream);
  if (e) return hipfail(c, e, "output gradient");
  return wnet_update(c, md, p, nt, w, lr, step, stream);
}

extern "C" int tm_set_weight_table(tm_ctx* c, const float* tab, int32_t nt, float xmax, void* stream) {
  if (!c) return TM_EINVAL;
  if (nt < 2 || nt > TM_WTAB_MAX) return fail(c, TM_EINVAL, "table points %d outside 2..%d", nt, TM_WTAB_MAX);
  if (!(xmax > 0.f) || !std::isfinite(xmax)) return fail(c, TM_EINVAL, "xmax must be > 0");
  if (!tab) return fail(c, TM_EINVAL, "tab is NULL");
  HIPCHK(c, hipSetDevice(c->device));
  void* dst = ws_get(c, WS_WTAB, (size_t)nt * 2 * sizeof(float));
  if (!dst) return fail(c, TM_ENOMEM, "table workspace");
  int e = tmk::launch_copy(dst, tab, (int64_t)nt * 2 * sizeof(float), stream);
  if (e) return hipfail(c, e, "table copy");
  c->wtab_n = nt;
  c->wtab_xmax = xmax;
  return TM_OK;
}

extern "C" int tm_retrieve_learned(tm_ctx* c, tm_dims d, const tm_c32* masks, const void* I, tm_c32* t,
                                   const tm_retrieve_opts* o, double rho_fallback, tm_row_stats* stats,
                                   int32_t* n_fallback, void* stream) {
  if (!c) return TM_EINVAL;
  if (!o) return fail(c, TM_EINVAL, "opts is NULL");
  if (o->start != TM_START_LEARNED) return fail(c, TM_EINVAL, "opts->start must be TM_START_LEARNED");
  if (!(rho_fallback >= 0.0)) return fail(c, TM_EINVAL, "rho_fallback must be >= 0");
  if (!n_fallback) return fail(c, TM_EINVAL, "n_fallback is NULL");
  *n_fallback = 0;
  tmk::row_launcher fn;
  int r = check_dims(c, d, &fn);
  if (r) return r;
  if (d.P == 0) return tm_retrieve(c, d, masks, I, t, o, stats, stream);
  if (!masks || !I || !t) return fail(c, TM_EINVAL, "null pointer argument");
  HIPCHK(c, hipSetDevice(c->device));
  const int N = d.n1 * d.n2;
  const size_t row = (size_t)N * sizeof(tm_c32);
  const size_t irow = (size_t)d.K * N * (o->I_dtype == TM_BF16 ? 2 : 4);
  void* seed = ws_get(c, WS_PH_BASE + 41, (size_t)d.P * row);
  tm_row_stats* st = stats ? stats : (tm_row_stats*)ws_get(c, WS_PH_BASE + 42, (size_t)d.P * sizeof(tm_row_stats));
  int* idx = (int*)ws_get(c, WS_PH_BASE + 43, (size_t)(d.P + 1) * sizeof(int));
  if (!seed || !st || !idx) return fail(c, TM_ENOMEM, "fallback workspace");
  int e = tmk::launch_copy(seed, t, (int64_t)d.P * row, stream);
  if (e) return hipfail(c, e, "seed copy");
  if ((r = tm_retrieve(c, d, masks, I, t, o, st, stream))) return r;
  // rows whose residual stays above rho_fallback are redone from the plain truncated start
  int* count = idx + d.P;
  if (!c->pinned) HIPCHK(c, hipHostMalloc((void**)&c->pinned, 8 * sizeof(double), hipHostMallocDefault));
  e = tmk::launch_fill_zero(count, sizeof(int), stream);
  if (!e) e = tmk::launch_flag_rows(st, d.P, rho_fallback, idx, count, stream);
  if (e) return hipfail(c, e, "flag rows");
  HIPCHK(c, hipMemcpyAsync(c->pinned, count, sizeof(int), hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
  const int nf = *(const int*)c->pinned;
  *n_fallback = nf;
  if (nf <= 0) return TM_OK;
  char* tf = (char*)ws_get(c, WS_PH_BASE + 44, (size_t)nf * row);
  char* If = (char*)ws_get(c, WS_PH_BASE + 45, (size_t)nf * irow);
  tm_row_stats* stf = (tm_row_stats*)ws_get(c, WS_PH_BASE + 46, (size_t)nf * sizeof(tm_row_stats));
  if (!tf || !If || !stf) return fail(c, TM_ENOMEM, "fallback workspace");
  // BF16 rows are K N 2-byte values: gather them as 8-byte words when K N is a multiple of 4
  if (irow % 8) return fail(c, TM_EUNSUPPORTED, "fallback rows of %zu bytes", irow);
  e = tmk::launch_gather_rows(tf, seed, idx, nf, (int64_t)row, stream);
  if (!e) e = tmk::launch_gather_rows(If, I, idx, nf, (int64_t)irow, stream);
  if (e) return hipfail(c, e, "fallback gather");
  tm_retrieve_opts fo = *o;
  fo.start = TM_START_LANCZOS;
  tm_dims df = d;
  df.P = nf;
  if ((r = tm_retrieve(c, df, masks, If, (tm_c32*)tf, &fo, stf, stream))) return r;
  e = tmk::launch_select_rows(t, tf, st, stf, idx, nf, (int64_t)row, stream);
  if (e) return hipfail(c, e, "fallback select");
  return TM_OK;
}
