// api.hip -- the C ABI of libpaid (declared in include/paid.h): argument
// checks, device workspace, the round loop of the adaptive scheme (Alg. 2)
// over all containers, and the diagnostic entry points.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "launch.h"
#include "paid.h"

using namespace paid;

namespace {

thread_local std::string g_create_error;

struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes <= n && p) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    size_t want = bytes ? bytes : 1;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) n = want;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

}  // namespace

struct paid_ctx {
  paid_config cfg;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // workspace
  DevBuf entries, tab, zeta, svals, ctr, qv, ffc;
  DevBuf code, key, Q, E;
  DevBuf slot_i, slot_d, sel, dv, de, dep, itau, errp, stl, counters, outs, errs;
  // learned seeding
  DevBuf seedw, sfeat, sfold, sy, sact, pyr, seedd, ifill, labtmp, rowsz, rperm, movei, upart;
  bool seed_on = false;
  int seed_dmax = 8;
  double seed_kappa = 2.0;
  float *feat_out = nullptr, *lab_out = nullptr;
  const double *pair_w = nullptr;  // weighted mode: caller's [n_ctr][M][M]
  DevBuf pairw;
  // lockstep mode (batch = batch_max = 1): creation index of every leaf
  DevBuf born;
  // leaf output of finished containers
  int *leaf_codes = nullptr;
  double *leaf_q = nullptr;
  long leaf_cap = 0;
  DevBuf lcodes, lq;
  int *host_counters = nullptr;  // pinned
  int max_J = 1;                 // rows of the largest table of the last build
  int lds_limit = 0;             // LDS bytes per workgroup (device attribute)
  float *noalloc = nullptr;      // this device's fixed working memory (paid_mlp_loss_grad_noalloc)
  // profile: around the evaluation launch of the two rounds in flight
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
  hipEvent_t evd[2] = {nullptr, nullptr};  // end of each of the two rounds in flight
};

namespace {

int fail(paid_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(paid_ctx *c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf; else g_create_error = buf;
  return code;
}

#define HIPCHK(ctx, expr)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      (void)hipGetLastError();                                                                \
      return fail(ctx, e_ == hipErrorOutOfMemory ? PAID_ENOMEM : PAID_EDEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                          \
    }                                                                                         \
  } while (0)

bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

constexpr double kPiH = 3.14159265358979323846;

// Clenshaw-Curtis rule with n intervals on [-1,1], ascending nodes; weights
// from the moment conditions sum_k w_k T_j(x_k) = int_{-1}^{1} T_j, j = 0..n,
// solved by Gaussian elimination (exact rule of interpolatory type).
void cc_rule_ascending(int n, double *x, double *w) {
  const double pi = 3.14159265358979323846;
  std::vector<double> A((n + 1) * (n + 2));
  for (int k = 0; k <= n; ++k) x[k] = sin(pi * (double)(2 * k - n) / (2.0 * n));
  for (int j = 0; j <= n; ++j) {
    for (int k = 0; k <= n; ++k) A[j * (n + 2) + k] = cos(j * acos(fmax(-1.0, fmin(1.0, x[k]))));
    A[j * (n + 2) + n + 1] = (j % 2) ? 0.0 : 2.0 / (1.0 - (double)j * j);
  }
  for (int c = 0; c <= n; ++c) {  // partial pivoting
    int piv = c;
    for (int r = c + 1; r <= n; ++r)
      if (fabs(A[r * (n + 2) + c]) > fabs(A[piv * (n + 2) + c])) piv = r;
    for (int k = 0; k < n + 2; ++k) std::swap(A[c * (n + 2) + k], A[piv * (n + 2) + k]);
    for (int r = 0; r <= n; ++r) {
      if (r == c) continue;
      double f = A[r * (n + 2) + c] / A[c * (n + 2) + c];
      for (int k = c; k < n + 2; ++k) A[r * (n + 2) + k] -= f * A[c * (n + 2) + k];
    }
  }
  for (int k = 0; k <= n; ++k) w[k] = A[k * (n + 2) + n + 1] / A[k * (n + 2) + k];
  for (int k = 0; k <= n / 2; ++k) {  // symmetrise
    double s = 0.5 * (w[k] + w[n - k]);
    w[k] = w[n - k] = s;
  }
}

int g_rule_ready[64] = {0};

// device address of each device's fixed working memory, looked up once per
// device with that device current
std::mutex g_noalloc_mu;
float *g_noalloc_ptr[64] = {nullptr};

int ensure_noalloc(paid_ctx *c) {
  const int dev = c->cfg.device;
  if (dev < 0 || dev >= 64) return fail(c, PAID_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    float *p = nullptr;
    HIPCHK(c, noalloc_scratch_address(&p));
    if (!p) return fail(c, PAID_EDEVICE, "no address for the fixed working memory");
    g_noalloc_ptr[dev] = p;
  }
  c->noalloc = g_noalloc_ptr[dev];
  return PAID_OK;
}

int ensure_rule(paid_ctx *c) {
  int dev = c->cfg.device;
  if (dev >= 0 && dev < 64 && g_rule_ready[dev]) return PAID_OK;
  RuleConst rc;
  double x1[kNCo];
  cc_rule_ascending(kNF - 1, rc.xi, rc.w2);
  cc_rule_ascending(kNCo - 1, x1, rc.w1);
  for (int d = 0; d < kDelDepths; ++d)
    for (int a = 0; a < 5; ++a) {
      const double del = ldexp(kPiH, -(d + 1)) * rc.xi[a];
      rc.cdel[d][a] = cos(del);
      rc.sdel[d][a] = sin(del);
    }
  HIPCHK(c, set_rule_constants(rc));
  if (dev >= 0 && dev < 64) g_rule_ready[dev] = 1;
  return PAID_OK;
}

// host bookkeeping of one parameter row's table (sizes only; the table
// itself is computed on the device)
Entry make_entry(const paid_params &p, int kind, int &off) {
  Entry e;
  memset(&e, 0, sizeof e);
  e.t = p.t;
  e.tp = p.tp;
  e.mu = p.mu;
  e.T = p.T;
  e.Om = p.Omega;
  e.kind = kind;
  e.emax = 4.0 * fabs(p.t) + 4.0 * fabs(p.tp) + fabs(p.mu);
  if (kind <= 1) {
    e.w = kPiH * p.T;
    e.inv_w = 1.0 / e.w;
    double top = e.emax * 1.01 + 1e-3 * e.w;
    e.J = tab_rows(top, e.w);
    double cJ, hJ;
    tab_interval(e.J - 1, e.w, cJ, hJ);
    double xJ = cJ + hJ;  // top of the last interval
    double big = fmax(fmax(p.Omega, 1.6 * xJ), kPiH * p.T);
    int nm = (int)ceil((4.0 * big / (kPiH * p.T) - 1.0) / 2.0);
    e.nmats = nm < 8 ? 8 : nm;
  } else {
    e.w = 1.0;
    e.inv_w = 1.0;
    e.J = 1;
    e.nmats = 0;
  }
  e.tab_off = off;
  off += e.J * kTabStride;
  return e;
}

// LDS bytes one workgroup may use on the context's device (queried once)
int lds_limit(paid_ctx *c) {
  if (c->lds_limit <= 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c->cfg.device) != hipSuccess ||
        v <= 0)
      v = 65536;
    c->lds_limit = v;
  }
  return c->lds_limit;
}

int build_tables(paid_ctx *c, const paid_params *params, int n, int kind) {
  std::vector<Entry> es(n);
  int off = 0, maxJ = 1;
  for (int i = 0; i < n; ++i) {
    es[i] = make_entry(params[i], kind, off);
    if (es[i].J > maxJ) maxJ = es[i].J;
  }
  HIPCHK(c, c->entries.ensure(sizeof(Entry) * n));
  HIPCHK(c, c->tab.ensure(sizeof(double) * (size_t)off));
  HIPCHK(c, c->zeta.ensure(sizeof(double) * (size_t)n * (kTabKTail + 1)));
  HIPCHK(c, c->svals.ensure(sizeof(double2) * (size_t)n * maxJ * kTabPts));
  HIPCHK(c, hipMemcpyAsync(c->entries.p, es.data(), sizeof(Entry) * n, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemsetAsync(c->tab.p, 0, sizeof(double) * (size_t)off, c->stream));
  TabArgs a;
  a.entries = c->entries.as<Entry>();
  a.n_entries = n;
  a.max_J = maxJ;
  c->max_J = maxJ;
  a.tab = c->tab.as<double>();
  a.zeta = c->zeta.as<double>();
  a.svals = c->svals.as<double2>();
  HIPCHK(c, launch_tables(a, c->stream));
  return PAID_OK;
}

int check_params(paid_ctx *c, const paid_params *p, int n, int kind) {
  for (int i = 0; i < n; ++i) {
    const paid_params &r = p[i];
    if (!isfinite(r.t) || !isfinite(r.tp) || !isfinite(r.mu) || !isfinite(r.T) ||
        !isfinite(r.Omega))
      return fail(c, PAID_EINVAL, "params[%d] not finite", i);
    if (kind <= 1 && !(r.T > 0.0)) return fail(c, PAID_EINVAL, "params[%d].T must be > 0", i);
    if (kind <= 1 && !(r.Omega >= 0.0)) return fail(c, PAID_EINVAL, "params[%d].Omega must be >= 0", i);
    if (kind <= 1 && r.T < 1e-6) return fail(c, PAID_EINVAL, "params[%d].T below 1e-6 is not supported", i);
  }
  return PAID_OK;
}

int check_ff(paid_ctx *c, const double *ff, int n_ff, int L, int &identity) {
  if (L < 0 || L > kMaxL) return fail(c, PAID_EINVAL, "ff_L must be 0..%d", kMaxL);
  int nb = (2 * L + 1) * (2 * L + 1);
  if (n_ff < 1 || n_ff > nb) return fail(c, PAID_EINVAL, "n_ff must be 1..%d", nb);
  identity = (n_ff == nb);
  for (int i = 0; i < n_ff; ++i)
    for (int j = 0; j < n_ff; ++j) {
      double s = 0.0;
      for (int k = 0; k < nb; ++k) s += ff[i * nb + k] * ff[j * nb + k];
      if (fabs(s - (i == j ? 1.0 : 0.0)) > 1e-12)
        return fail(c, PAID_EINVAL, "form factors not orthonormal (row %d, %d)", i, j);
    }
  for (int i = 0; i < n_ff && identity; ++i)
    for (int k = 0; k < nb; ++k)
      if (ff[i * nb + k] != (i == k ? 1.0 : 0.0)) identity = 0;
  return PAID_OK;
}

// host copy of an input array that may live on the device
template <class T>
int to_host(paid_ctx *c, const T *p, size_t n, std::vector<T> &out) {
  out.resize(n);
  if (n == 0) return PAID_OK;
  if (is_device_ptr(p)) {
    HIPCHK(c, hipMemcpy(out.data(), p, sizeof(T) * n, hipMemcpyDeviceToHost));
  } else {
    memcpy(out.data(), p, sizeof(T) * n);
  }
  return PAID_OK;
}

// device view of a caller array: the pointer itself, or a staged copy in tmp
template <class T>
int stage_in(paid_ctx *c, const T *p, size_t n, DevBuf &tmp, const T *&d) {
  if (is_device_ptr(p)) {
    d = p;
    return PAID_OK;
  }
  HIPCHK(c, tmp.ensure(sizeof(T) * (n ? n : 1)));
  if (n) HIPCHK(c, hipMemcpyAsync(tmp.p, p, sizeof(T) * n, hipMemcpyHostToDevice, c->stream));
  d = tmp.as<T>();
  return PAID_OK;
}

// device buffer for a caller output: the pointer itself, or tmp (copied back
// with finish_out)
template <class T>
int stage_out(paid_ctx *c, T *p, size_t n, DevBuf &tmp, T *&d) {
  if (is_device_ptr(p)) {
    d = p;
    return PAID_OK;
  }
  HIPCHK(c, tmp.ensure(sizeof(T) * (n ? n : 1)));
  d = tmp.as<T>();
  return PAID_OK;
}

template <class T>
int finish_out(paid_ctx *c, T *p, const T *d, size_t n) {
  if (p != d && n) HIPCHK(c, hipMemcpyAsync(p, d, sizeof(T) * n, hipMemcpyDeviceToHost, c->stream));
  return PAID_OK;
}

// the full set of per-sample training buffers for n samples, carved from buf
int carve_act(paid_ctx *c, DevBuf &buf, int n, MlpAct &a, float *&yhat, float *&dY) {
  const size_t h = (size_t)kMlpHid * n, o = (size_t)kMlpOut * n;
  HIPCHK(c, buf.ensure(sizeof(float) * (9 * h + 2 * o)));
  float *p = buf.as<float>();
  for (int l = 0; l < 3; ++l) {
    a.Z[l] = p + (size_t)l * h;
    a.A[l] = p + (size_t)(3 + l) * h;
    a.D[l] = p + (size_t)(6 + l) * h;
  }
  a.Z[3] = nullptr;
  yhat = p + 9 * h;
  dY = yhat + o;
  return PAID_OK;
}

struct SlotLayout {  // carving of the small per-slot arrays
  int *cid, *state, *nleaf, *selcnt, *woff, *flags, *depth;
};

}  // namespace

extern "C" {

int paid_config_default(paid_config *cfg) {
  if (!cfg) return PAID_EINVAL;
  memset(cfg, 0, sizeof *cfg);
  cfg->device = 0;
  cfg->N = 4;
  cfg->batch = 8;
  cfg->batch_max = 1024;
  cfg->err_mode = PAID_ERR_GLOBAL;
  cfg->precision = PAID_FP64;
  cfg->gram = PAID_GRAM_SEPARABLE;
  cfg->kind = PAID_BUBBLE_DOT;
  cfg->nu = 1e-3;
  cfg->max_regions = 1L << 18;
  cfg->max_active = 0;
  cfg->pool_gib = 0.0;
  cfg->gauss[2] = 1.0;
  cfg->stream = nullptr;
  return PAID_OK;
}

int paid_create(paid_ctx **out, const paid_config *cfg_in) {
  if (!out) return fail(nullptr, PAID_EINVAL, "out is NULL");
  *out = nullptr;
  paid_config cfg;
  if (cfg_in) cfg = *cfg_in; else paid_config_default(&cfg);
  if (cfg.N != 4) return fail(nullptr, PAID_EINVAL, "only N = 4 is implemented");
  if (cfg.batch < 1 || cfg.batch_max < cfg.batch)
    return fail(nullptr, PAID_EINVAL, "need 1 <= batch <= batch_max");
  if (cfg.err_mode != PAID_ERR_GLOBAL && cfg.err_mode != PAID_ERR_PER_INTEGRAL &&
      cfg.err_mode != PAID_ERR_WEIGHTED)
    return fail(nullptr, PAID_EINVAL, "bad err_mode");
  if (cfg.precision != PAID_FP64 && cfg.precision != PAID_FP32 && cfg.precision != PAID_BF16X3)
    return fail(nullptr, PAID_EINVAL, "bad precision");
  if (cfg.precision != PAID_FP64 && cfg.gram != PAID_GRAM_MFMA)
    return fail(nullptr, PAID_EINVAL, "reduced precision needs the matrix-core projection");
  if (cfg.gram != PAID_GRAM_MFMA && cfg.gram != PAID_GRAM_SEPARABLE)
    return fail(nullptr, PAID_EINVAL, "bad gram mode");
  if (cfg.kind < 0 || cfg.kind > 3) return fail(nullptr, PAID_EINVAL, "bad kind");
  if (cfg.kind == PAID_GAUSS && !(cfg.gauss[2] > 0)) return fail(nullptr, PAID_EINVAL, "gauss width must be > 0");
  if (cfg.small_regions < 0 || (cfg.small_regions > 0 && cfg.small_regions < 16))
    return fail(nullptr, PAID_EINVAL, "small_regions must be 0 or >= 16");
  if (cfg.big_share < 0 || cfg.big_share >= 1) return fail(nullptr, PAID_EINVAL, "big_share must lie in [0, 1)");
  if (cfg.max_regions < 16 || cfg.max_regions > (1L << 28))
    return fail(nullptr, PAID_EINVAL, "max_regions must be in [16, 2^28]");
  if (!(cfg.nu >= 0)) return fail(nullptr, PAID_EINVAL, "nu must be >= 0");
  if (cfg.eval_wg_per_cu < 0 || cfg.eval_wg_per_cu > 1024)
    return fail(nullptr, PAID_EINVAL, "eval_wg_per_cu must be 0..1024");
  if (cfg.symmetry != 0 && cfg.symmetry != 1) return fail(nullptr, PAID_EINVAL, "symmetry must be 0 or 1");
  if (cfg.eval_layout != 0 && cfg.eval_layout != 1) return fail(nullptr, PAID_EINVAL, "eval_layout must be 0 or 1");
  if (cfg.symmetry && cfg.kind == PAID_GAUSS)
    return fail(nullptr, PAID_EINVAL, "the Gaussian test integrand is not even under p -> -p");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(nullptr, PAID_EDEVICE, "no HIP device");
  if (cfg.device < 0 || cfg.device >= ndev) return fail(nullptr, PAID_EINVAL, "bad device ordinal");
  e = hipSetDevice(cfg.device);
  if (e != hipSuccess) return fail(nullptr, PAID_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  paid_ctx *c = new paid_ctx();
  c->cfg = cfg;
  if (cfg.stream) {
    c->stream = (hipStream_t)cfg.stream;
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return fail(nullptr, PAID_EDEVICE, "stream: %s", hipGetErrorString(e));
    }
    c->own_stream = true;
  }
  e = hipHostMalloc((void **)&c->host_counters, 64, hipHostMallocDefault);
  if (e != hipSuccess) {
    paid_destroy(c);
    return fail(nullptr, PAID_ENOMEM, "pinned counters: %s", hipGetErrorString(e));
  }
  if (cfg.profile) {
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreate(&c->ev2) != hipSuccess || hipEventCreate(&c->ev3) != hipSuccess) {
      paid_destroy(c);
      return fail(nullptr, PAID_EDEVICE, "hipEventCreate failed");
    }
  }
  for (int k = 0; k < 2; ++k)
    if (hipEventCreateWithFlags(&c->evd[k], hipEventDisableTiming) != hipSuccess) {
      paid_destroy(c);
      return fail(nullptr, PAID_EDEVICE, "hipEventCreate failed");
    }
  int rc = ensure_rule(c);
  if (rc == PAID_OK) rc = ensure_noalloc(c);
  if (rc != PAID_OK) {
    g_create_error = c->err;
    paid_destroy(c);
    return rc;
  }
  *out = c;
  return PAID_OK;
}

void paid_destroy(paid_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->cfg.device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  DevBuf *bufs[] = {&c->entries, &c->tab,  &c->zeta,  &c->svals, &c->ctr,   &c->qv,
                    &c->ffc,     &c->code, &c->key,   &c->Q,     &c->E,     &c->slot_i,
                    &c->slot_d,  &c->sel,  &c->dv,    &c->de,    &c->dep,   &c->itau,
                    &c->errp,    &c->stl,  &c->counters, &c->outs, &c->errs,
                    &c->seedw,   &c->sfeat, &c->sfold, &c->sy,  &c->sact,  &c->pyr,
                    &c->seedd,   &c->ifill, &c->labtmp, &c->pairw, &c->born, &c->lcodes,
                    &c->lq,      &c->rowsz, &c->rperm, &c->movei, &c->upart};
  for (DevBuf *b : bufs) b->release();
  if (c->host_counters) (void)hipHostFree(c->host_counters);
  for (hipEvent_t ev : {c->ev0, c->ev1, c->ev2, c->ev3, c->evd[0], c->evd[1]})
    if (ev) (void)hipEventDestroy(ev);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char *paid_last_error(const paid_ctx *c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

int paid_integrate(paid_ctx *c, const paid_params *params, int n_params, const double *q,
                   int n_q, const double *ff, int n_ff, int ff_L, unsigned channels, double rtol,
                   double atol, double *out, double *err_out, paid_stats *stats) {
  auto t0 = std::chrono::steady_clock::now();
  if (!c) return PAID_EINVAL;
  c->err.clear();
  if (!params || !q || !ff || !out) return fail(c, PAID_EINVAL, "NULL input or output");
  if (n_params < 1 || n_q < 1) return fail(c, PAID_EINVAL, "n_params and n_q must be >= 1");
  if ((channels & ~3u) || !(channels & 3u)) return fail(c, PAID_EINVAL, "channels must be PAID_PP | PAID_PH");
  if (!(rtol >= 0) || !(atol >= 0) || !(rtol > 0 || atol > 0))
    return fail(c, PAID_EINVAL, "need rtol > 0 or atol > 0 (both >= 0)");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  const paid_config &cfg = c->cfg;
  std::vector<paid_params> hp;
  std::vector<double> hq, hff;
  int rc;
  if ((rc = to_host(c, params, (size_t)n_params, hp)) != PAID_OK) return rc;
  if ((rc = to_host(c, q, (size_t)n_q * 2, hq)) != PAID_OK) return rc;
  int nb = (2 * ff_L + 1) * (2 * ff_L + 1);
  if (ff_L < 0 || ff_L > kMaxL) return fail(c, PAID_EINVAL, "ff_L must be 0..%d", kMaxL);
  if (n_ff < 1 || n_ff > nb) return fail(c, PAID_EINVAL, "n_ff must be 1..%d", nb);
  if ((rc = to_host(c, ff, (size_t)n_ff * nb, hff)) != PAID_OK) return rc;
  for (double v : hq)
    if (!isfinite(v)) return fail(c, PAID_EINVAL, "q not finite");
  if ((rc = check_params(c, hp.data(), n_params, cfg.kind)) != PAID_OK) return rc;
  int identity = 0;
  if ((rc = check_ff(c, hff.data(), n_ff, ff_L, identity)) != PAID_OK) return rc;

  const int n_ch = ((channels & 1u) ? 1 : 0) + ((channels & 2u) ? 1 : 0);
  const int ch_first = (channels & 1u) ? 0 : 1;
  const long n_ctr_l = (long)n_params * n_q * n_ch;
  if (n_ctr_l > (1L << 30)) return fail(c, PAID_EINVAL, "too many containers");
  const int n_ctr = (int)n_ctr_l;
  const int M = n_ff, MU = M * (M + 1) / 2;
  const bool store_E = (err_out != nullptr) || cfg.err_mode == PAID_ERR_PER_INTEGRAL;

  // tables and container constants
  if ((rc = build_tables(c, hp.data(), n_params, cfg.kind)) != PAID_OK) return rc;
  HIPCHK(c, c->qv.ensure(sizeof(double) * 2 * n_q));
  HIPCHK(c, hipMemcpyAsync(c->qv.p, hq.data(), sizeof(double) * 2 * n_q, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, c->ffc.ensure(sizeof(double) * n_ff * nb));
  HIPCHK(c, hipMemcpyAsync(c->ffc.p, hff.data(), sizeof(double) * n_ff * nb, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, c->ctr.ensure(sizeof(Ctr) * n_ctr));
  HIPCHK(c, launch_container_setup(c->ctr.as<Ctr>(), n_ctr, c->qv.as<double>(), n_q, n_ch, ch_first, c->stream));

  // pool: slots x capacity; with small_regions, large slots (capb) first,
  // then small ones (cap)
  const long capb = cfg.max_regions;
  const bool two = cfg.small_regions > 0 && cfg.small_regions < capb;
  const long cap = two ? cfg.small_regions : capb;
  const size_t rec = 16 + 8 * (size_t)MU + (store_E ? 4 * (size_t)MU : 0);
  size_t pool_bytes, rest_bytes = 0;  // rest: for the per-slot round buffers (0: unchecked)
  if (cfg.pool_gib > 0) {
    pool_bytes = (size_t)(cfg.pool_gib * 1073741824.0);
  } else {
    size_t fr = 0, tot = 0;
    HIPCHK(c, hipMemGetInfo(&fr, &tot));
    const double avail = (double)(fr + c->code.n + c->key.n + c->Q.n + c->E.n + c->dv.n + c->dep.n);
    pool_bytes = (size_t)(0.55 * avail);
    rest_bytes = (size_t)(0.35 * avail);
  }
  long Wb = 0;
  if (two) {
    const double share = cfg.big_share > 0 ? cfg.big_share : 0.25;
    Wb = (long)(share * (double)pool_bytes / ((double)capb * rec));
    if (Wb < 1) Wb = 1;
    if (Wb > n_ctr) Wb = n_ctr;
  }
  const size_t big_bytes = (size_t)Wb * capb * rec;
  long Ws = cfg.max_active > 0 ? cfg.max_active - Wb
                               : (pool_bytes > big_bytes ? (long)((pool_bytes - big_bytes) / ((size_t)cap * rec)) : 0);
  if (Ws > n_ctr) Ws = n_ctr;
  if (Wb + Ws > 65536) Ws = 65536 - Wb;
  // the round buffers of every slot (deltas, selections) must fit beside the pool
  const size_t slot_rest = (size_t)cfg.batch_max * (8 * (size_t)MU * (store_E ? 2 : 1) + 16) + 32 * (size_t)MU;
  if (rest_bytes > 0 && (size_t)(Wb + Ws) * slot_rest > rest_bytes) Ws = (long)(rest_bytes / slot_rest) - Wb;
  if (Ws < 1) return fail(c, PAID_ENOMEM, "region pool too small for one container of %ld regions", cap);
  const long W = Wb + Ws;
  const size_t regions = (size_t)Wb * capb + (size_t)Ws * cap;
  const int bmax = cfg.batch_max, bmin = cfg.batch;
  HIPCHK(c, c->code.ensure(sizeof(uint64_t) * regions));
  HIPCHK(c, c->key.ensure(sizeof(double) * regions));
  HIPCHK(c, c->Q.ensure(sizeof(double) * regions * MU));
  if (store_E) HIPCHK(c, c->E.ensure(sizeof(float) * regions * MU));
  HIPCHK(c, c->movei.ensure(sizeof(int) * (size_t)(W + Wb + 1)));
  HIPCHK(c, c->upart.ensure(sizeof(double) * update_scratch_doubles((int)W, MU)));
  HIPCHK(c, c->slot_i.ensure(sizeof(int) * (8 * W + 8)));
  HIPCHK(c, c->slot_d.ensure(sizeof(double) * (W * (size_t)MU + W)));
  HIPCHK(c, c->errp.ensure(sizeof(double) * W * (size_t)MU));
  HIPCHK(c, c->itau.ensure(sizeof(float) * W * (size_t)MU));
  HIPCHK(c, c->sel.ensure(sizeof(int) * W * (size_t)bmax));
  HIPCHK(c, c->dv.ensure(sizeof(double) * W * (size_t)bmax * MU));
  HIPCHK(c, c->de.ensure(sizeof(double) * W * (size_t)bmax));
  if (store_E) HIPCHK(c, c->dep.ensure(sizeof(double) * W * (size_t)bmax * MU));
  HIPCHK(c, c->stl.ensure(sizeof(long) * 3 * W));
  HIPCHK(c, c->ifill.ensure(sizeof(int) * W * (size_t)bmax));
  const bool lockstep = bmin == 1 && bmax == 1;
  if (lockstep) HIPCHK(c, c->born.ensure(sizeof(unsigned int) * regions));
  HIPCHK(c, c->counters.ensure(256));
  const bool out_dev = is_device_ptr(out), err_dev = err_out && is_device_ptr(err_out);
  const size_t out_bytes = sizeof(double) * (size_t)n_ctr * M * M;
  if (!out_dev) HIPCHK(c, c->outs.ensure(out_bytes));
  if (err_out && !err_dev) HIPCHK(c, c->errs.ensure(out_bytes));

  Problem P;
  memset(&P, 0, sizeof P);
  P.entries = c->entries.as<Entry>();
  P.tab = c->tab.as<double>();
  P.tab_rows = c->max_J;
  P.lds_limit = lds_limit(c);
  P.ctr = c->ctr.as<Ctr>();
  P.n_ctr = n_ctr;
  P.kind = cfg.kind;
  P.err_mode = cfg.err_mode;
  P.precision = cfg.precision;
  P.gram = cfg.gram;
  P.gauss_x = cfg.gauss[0];
  P.gauss_y = cfg.gauss[1];
  P.gauss_s = cfg.gauss[2];
  P.rtol = rtol;
  P.atol = atol;
  P.nu = cfg.nu;
  P.L = ff_L;
  P.nb = 2 * ff_L + 1;
  P.MB = nb;
  P.M = M;
  P.MU = MU;
  P.ff_identity = identity;
  P.eval_layout = cfg.eval_layout;
  if (eval_lds_bytes(P) == 0)
    return fail(c, PAID_EINVAL, "frequency-sum table of %d rows does not fit in LDS (T too small against the band)",
                P.tab_rows);
  P.ffc = c->ffc.as<double>();
  P.W = (int)W;
  P.cap = cap;
  P.Wb = (int)Wb;
  P.capb = capb;
  P.moveq = c->movei.as<int>();
  P.upart = c->upart.as<double>();
  P.promo = P.moveq + W;
  P.bmin = bmin;
  P.bmax = bmax;
  P.code = c->code.as<uint64_t>();
  P.key = c->key.as<double>();
  P.Q = c->Q.as<double>();
  P.E = store_E ? c->E.as<float>() : nullptr;
  int *si = c->slot_i.as<int>();
  P.cid = si;
  P.state = si + W;
  P.nleaf = si + 2 * W;
  P.selcnt = si + 3 * W;
  P.flags = si + 4 * W;
  P.st_depth = si + 5 * W;
  P.woff = si + 6 * W;  // W + 1 entries
  P.sel = c->sel.as<int>();
  P.val = c->slot_d.as<double>();
  P.err = c->slot_d.as<double>() + W * (size_t)MU;
  P.errp = store_E ? c->errp.as<double>() : nullptr;
  P.itau = c->itau.as<float>();
  P.dv = c->dv.as<double>();
  P.de = c->de.as<double>();
  P.dep = store_E ? c->dep.as<double>() : nullptr;
  P.st_rounds = c->stl.as<long>();
  P.st_splits = c->stl.as<long>() + W;
  P.st_evals = c->stl.as<long>() + 2 * W;
  P.ifill = c->ifill.as<int>();
  int *cnt = c->counters.as<int>();
  P.qhead = cnt;            // [0]
  P.counters = cnt + 4;     // [4..7]: done, not converged, work items
  P.gstats = reinterpret_cast<long long *>(cnt + 16);  // [16..23]
  P.out = out_dev ? out : c->outs.as<double>();
  P.born = lockstep ? c->born.as<unsigned int>() : nullptr;
  int *lcodes_dev = nullptr;
  double *lq_dev = nullptr;
  const size_t nlc = (size_t)n_ctr * (size_t)c->leaf_cap;
  if (c->leaf_codes) {
    int rl;
    if ((rl = stage_out(c, c->leaf_codes, nlc * 3, c->lcodes, lcodes_dev)) != PAID_OK) return rl;
    if ((rl = stage_out(c, c->leaf_q, nlc * MU, c->lq, lq_dev)) != PAID_OK) return rl;
    P.leaf_codes = lcodes_dev;
    P.leaf_q = lq_dev;
    P.leaf_cap = c->leaf_cap;
  }
  P.err_out = err_out ? (err_dev ? err_out : c->errs.as<double>()) : nullptr;

  HIPCHK(c, hipMemsetAsync(c->slot_i.p, 0, sizeof(int) * (8 * W + 8), c->stream));
  HIPCHK(c, hipMemsetAsync(c->counters.p, 0, 256, c->stream));
  HIPCHK(c, hipMemsetAsync(c->stl.p, 0, sizeof(long) * 3 * W, c->stream));

  if (cfg.err_mode == PAID_ERR_WEIGHTED) {
    if (!c->pair_w) return fail(c, PAID_EINVAL, "PAID_ERR_WEIGHTED needs paid_set_pair_weights");
    const size_t nw = (size_t)n_ctr * M * M;
    const double *dw;
    int rw;
    if ((rw = stage_in(c, c->pair_w, nw, c->pairw, dw)) != PAID_OK) return rw;
    std::vector<double> hw;
    if ((rw = to_host(c, c->pair_w, nw, hw)) != PAID_OK) return rw;
    for (size_t i = 0; i < nw; ++i)
      if (!(hw[i] >= 0.0) || !std::isfinite(hw[i])) return fail(c, PAID_EINVAL, "pair weight %zu not finite and >= 0", i);
    P.pair_w = dw;
  }

  // learned seeding: model features of every container, then the model
  const bool want_labels = c->lab_out != nullptr || c->feat_out != nullptr;
  if (cfg.symmetry && (c->seed_on || want_labels))
    return fail(c, PAID_EINVAL, "the half-zone mode takes neither a seed model nor tree labels");
  P.sym = cfg.symmetry;
  double seed_s = 0.0;
  if (c->seed_on || want_labels) {
    auto ts = std::chrono::steady_clock::now();
    HIPCHK(c, c->sfeat.ensure(sizeof(float) * kMlpIn * (size_t)n_ctr));
    HIPCHK(c, c->sfold.ensure(sizeof(int) * (size_t)n_ctr));
    HIPCHK(c, launch_seed_features(c->entries.as<Entry>(), c->qv.as<double>(), n_ctr, n_q, n_ch,
                                   ch_first, c->sfeat.as<float>(), c->sfold.as<int>(), c->stream));
    P.seed_fold = c->sfold.as<int>();
    if (c->seed_on) {
      HIPCHK(c, c->sy.ensure(sizeof(float) * kMlpOut * (size_t)n_ctr));
      const int chunk = n_ctr < 65536 ? n_ctr : 65536;
      HIPCHK(c, c->sact.ensure(sizeof(float) * 2 * kMlpHid * (size_t)chunk));
      MlpAct a;
      memset(&a, 0, sizeof a);
      a.A[0] = c->sact.as<float>();
      a.A[1] = a.A[0] + (size_t)kMlpHid * chunk;
      a.A[2] = a.A[0];
      for (int o = 0; o < n_ctr; o += chunk) {
        int nn = n_ctr - o < chunk ? n_ctr - o : chunk;
        HIPCHK(c, mlp_forward(c->seedw.as<float>(), c->sfeat.as<float>() + (size_t)o * kMlpIn, nn, a,
                              c->sy.as<float>() + (size_t)o * kMlpOut, c->stream));
      }
      HIPCHK(c, c->pyr.ensure(sizeof(double) * kPyr * (size_t)W));
      HIPCHK(c, c->seedd.ensure(sizeof(int) * (size_t)W));
      P.seed_y = c->sy.as<float>();
      P.pyr = c->pyr.as<double>();
      P.seed_d = c->seedd.as<int>();
      P.seed_dmax = c->seed_dmax;
      P.seed_thresh = 4.0 * c->seed_kappa;
      P.seed_limit = cap / 4;  // a seed tree fits a small slot
      // admission order: the parameter rows by predicted leaves, largest
      // first (ties by row), so that the deepest trees start early and the
      // call does not end on a few of them; each row's containers stay
      // together (one table per run of slots in the evaluation kernel)
      const int per_row = n_q * n_ch;
      HIPCHK(c, c->rowsz.ensure(sizeof(double) * (size_t)n_params));
      HIPCHK(c, c->rperm.ensure(sizeof(int) * (size_t)n_params));
      HIPCHK(c, launch_seed_rowsize(c->sy.as<float>(), n_params, per_row, c->rowsz.as<double>(), c->stream));
      std::vector<double> rsz(n_params);
      HIPCHK(c, hipMemcpyAsync(rsz.data(), c->rowsz.p, sizeof(double) * n_params, hipMemcpyDeviceToHost,
                               c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      std::vector<int> perm(n_params);
      for (int r = 0; r < n_params; ++r) {
        perm[r] = r;
        if (!(rsz[r] >= 0.0)) rsz[r] = 0.0;  // a model output that is not a number orders last
      }
      std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return rsz[a] > rsz[b]; });
      HIPCHK(c, hipMemcpyAsync(c->rperm.p, perm.data(), sizeof(int) * n_params, hipMemcpyHostToDevice,
                               c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      P.row_perm = c->rperm.as<int>();
      P.per_row = per_row;
    }
    if (c->lab_out) {
      if (is_device_ptr(c->lab_out)) {
        P.labels = c->lab_out;
      } else {
        HIPCHK(c, c->labtmp.ensure(sizeof(float) * kMlpOut * (size_t)n_ctr));
        P.labels = c->labtmp.as<float>();
      }
    }
    seed_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count();
  }

  int dev_cus = 256;
  {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, cfg.device) == hipSuccess && v > 0)
      dev_cus = v;
  }
  // guided partition over the workgroups resident at once; the default grid
  // (16 per resident slot) covers 4 e^16 work items per launch before its
  // last workgroup has to take a remainder of more than four
  const int occ = eval_occupancy(P);
  P.eval_slots = occ * dev_cus;
  const int eval_grid = dev_cus * (cfg.eval_wg_per_cu > 0 ? cfg.eval_wg_per_cu : 16 * occ);
  long rounds = 0, eval_items = 0;
  double eval_ms = 0.0;
  // one device round in three parts: admission, roots, selection and work
  // list; evaluation; updates, finalisation and the read-back of the three
  // counters the host needs (into one of two pinned buffers: parts 2 and 3
  // are the third part with buffer 0 and 1)
  auto part = [&](int k, hipStream_t st) -> hipError_t {
    hipError_t e;
    if (k == 0) {
      if ((e = launch_move(P, st)) != hipSuccess) return e;
      if ((e = launch_admit(P, st)) != hipSuccess) return e;
      if ((e = launch_root(P, st)) != hipSuccess) return e;
      if ((e = launch_select(P, st)) != hipSuccess) return e;
      return launch_worklist(P, st);
    }
    if (k == 1) return launch_eval(P, eval_grid, st);
    if ((e = launch_update(P, st)) != hipSuccess) return e;
    if ((e = launch_finalize(P, st)) != hipSuccess) return e;
    return hipMemcpyAsync(c->host_counters + 4 * (k - 2), cnt + 4, 12, hipMemcpyDeviceToHost, st);
  };
  // with cfg.graph each part is captured once and replayed every round (the
  // arguments of every launch are the same in every round); the profiling
  // events are recorded between the parts, outside the graphs
  hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
  struct GraphGuard {
    hipGraphExec_t *ge;
    ~GraphGuard() {
      for (int k = 0; k < 4; ++k)
        if (ge[k]) (void)hipGraphExecDestroy(ge[k]);
    }
  } gguard{gexec};
  if (cfg.graph) {
    for (int k = 0; k < 4; ++k) {
      hipGraph_t g = nullptr;
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
      hipError_t e1 = part(k, c->stream);
      hipError_t e2 = hipStreamEndCapture(c->stream, &g);
      if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        HIPCHK(c, e1 != hipSuccess ? e1 : e2);
      }
      hipError_t e3 = hipGraphInstantiate(&gexec[k], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCHK(c, e3);
    }
  }
  auto run_part = [&](int k) -> hipError_t {
    return gexec[k] ? hipGraphLaunch(gexec[k], c->stream) : part(k, c->stream);
  };
  // Two rounds in flight: round r + 1 is queued before the host reads the
  // counters of round r, so the device does not wait for the host between
  // rounds.  A round queued after the last one finds nothing to do (no
  // container left to admit, select or update).
  hipEvent_t evb[2] = {c->ev0, c->ev2}, eve[2] = {c->ev1, c->ev3};
  auto launch_round = [&](int buf) -> hipError_t {
    hipError_t e;
    if ((e = run_part(0)) != hipSuccess) return e;
    if (cfg.profile && (e = hipEventRecord(evb[buf], c->stream)) != hipSuccess) return e;
    if ((e = run_part(1)) != hipSuccess) return e;
    if (cfg.profile && (e = hipEventRecord(eve[buf], c->stream)) != hipSuccess) return e;
    if ((e = run_part(2 + buf)) != hipSuccess) return e;
    return hipEventRecord(c->evd[buf], c->stream);
  };
  HIPCHK(c, launch_round(0));
  int last = 0;  // buffer of the last round read
  for (long r = 0;; ++r) {
    const int buf = (int)(r & 1);
    HIPCHK(c, launch_round(buf ^ 1));
    HIPCHK(c, hipEventSynchronize(c->evd[buf]));
    const int *hc = c->host_counters + 4 * buf;
    last = buf;
    ++rounds;
    eval_items += hc[2];
    if (cfg.profile) {
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, evb[buf], eve[buf]));
      eval_ms += ms;
    }
    if (hc[0] >= n_ctr) break;
    if (rounds > 4L * capb + 64L * (n_ctr / Ws + 1)) {
      (void)hipStreamSynchronize(c->stream);
      return fail(c, PAID_EINTERNAL, "round loop did not finish (%ld rounds)", rounds);
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));  // the round queued after the last
  if (!out_dev) HIPCHK(c, hipMemcpyAsync(out, c->outs.p, out_bytes, hipMemcpyDeviceToHost, c->stream));
  if (err_out && !err_dev)
    HIPCHK(c, hipMemcpyAsync(err_out, c->errs.p, out_bytes, hipMemcpyDeviceToHost, c->stream));
  if (c->feat_out)
    HIPCHK(c, hipMemcpyAsync(c->feat_out, c->sfeat.p, sizeof(float) * kMlpIn * (size_t)n_ctr,
                             hipMemcpyDefault, c->stream));
  if (c->leaf_codes) {
    if ((rc = finish_out(c, c->leaf_codes, lcodes_dev, nlc * 3)) != PAID_OK) return rc;
    if ((rc = finish_out(c, c->leaf_q, lq_dev, nlc * MU)) != PAID_OK) return rc;
  }
  if (c->lab_out && P.labels != c->lab_out)
    HIPCHK(c, hipMemcpyAsync(c->lab_out, P.labels, sizeof(float) * kMlpOut * (size_t)n_ctr,
                             hipMemcpyDefault, c->stream));
  long long gs[5] = {0, 0, 0, 0, 0};
  HIPCHK(c, hipMemcpyAsync(gs, P.gstats, sizeof gs, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int notconv = c->host_counters[4 * last + 1];
  if (stats) {
    memset(stats, 0, sizeof *stats);
    stats->containers = n_ctr;
    stats->not_converged = notconv;
    stats->rounds = gs[0];
    stats->splits = gs[1];
    stats->regions = gs[2];
    stats->max_depth = (int)gs[3];
    stats->kernel_evals = gs[4];
    stats->launch_rounds = rounds;
    stats->max_active = (int)W;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->eval_seconds = eval_ms * 1e-3;
    stats->eval_launches = cfg.profile ? rounds : 0;
    stats->eval_items = eval_items;
    stats->seeded = c->seed_on ? n_ctr : 0;
    stats->seed_seconds = seed_s;
  }
  return notconv ? PAID_ENOCONV : PAID_OK;
}

int paid_kernel_eval(paid_ctx *c, const paid_params *p, unsigned channel, const double *a,
                     const double *b, int n, double *out) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  if (!p || n < 0 || (n > 0 && (!a || !b || !out))) return fail(c, PAID_EINVAL, "bad arguments");
  if (channel != PAID_PP && channel != PAID_PH) return fail(c, PAID_EINVAL, "channel must be PAID_PP or PAID_PH");
  if (c->cfg.kind > 1) return fail(c, PAID_EINVAL, "kernel_eval needs a bubble kind");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  std::vector<paid_params> hp;
  std::vector<double> ha, hb;
  int rc;
  if ((rc = to_host(c, p, 1, hp)) != PAID_OK) return rc;
  if ((rc = check_params(c, hp.data(), 1, c->cfg.kind)) != PAID_OK) return rc;
  if (n == 0) return PAID_OK;
  if ((rc = to_host(c, a, (size_t)n, ha)) != PAID_OK) return rc;
  if ((rc = to_host(c, b, (size_t)n, hb)) != PAID_OK) return rc;
  double emax = 4.0 * fabs(hp[0].t) + 4.0 * fabs(hp[0].tp) + fabs(hp[0].mu);
  for (int i = 0; i < n; ++i)
    if (!(fabs(ha[i]) <= emax && fabs(hb[i]) <= emax))
      return fail(c, PAID_EINVAL, "energy %d outside the dispersion range +-%g", i, emax);
  if ((rc = build_tables(c, hp.data(), 1, c->cfg.kind)) != PAID_OK) return rc;
  DevBuf tmp;
  HIPCHK(c, tmp.ensure(sizeof(double) * 3 * (size_t)n));
  double *da = tmp.as<double>(), *db = da + n, *dout = db + n;
  HIPCHK(c, hipMemcpyAsync(da, ha.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(db, hb.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_kernel_eval(c->entries.as<Entry>(), c->tab.as<double>(), channel == PAID_PH ? 1 : 0,
                               da, db, n, dout, c->stream));
  HIPCHK(c, hipMemcpyAsync(out, dout, sizeof(double) * n, hipMemcpyDefault, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  tmp.release();
  return PAID_OK;
}

int paid_children_eval(paid_ctx *c, const paid_params *p, const double *l, unsigned channel,
                       const double *ff, int n_ff, int ff_L, const int *codes, int n, double *q2n,
                       double *err) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  if (!p || !l || !ff || !codes || !q2n || !err || n < 1)
    return fail(c, PAID_EINVAL, "bad arguments");
  if (channel != PAID_PP && channel != PAID_PH) return fail(c, PAID_EINVAL, "channel must be PAID_PP or PAID_PH");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  const paid_config &cfg = c->cfg;
  std::vector<paid_params> hp;
  std::vector<double> hl, hff;
  std::vector<int> hc;
  int rc;
  if ((rc = to_host(c, p, 1, hp)) != PAID_OK) return rc;
  if ((rc = check_params(c, hp.data(), 1, cfg.kind)) != PAID_OK) return rc;
  if ((rc = to_host(c, l, 2, hl)) != PAID_OK) return rc;
  if (ff_L < 0 || ff_L > kMaxL) return fail(c, PAID_EINVAL, "ff_L must be 0..%d", kMaxL);
  int nb = (2 * ff_L + 1) * (2 * ff_L + 1);
  if (n_ff < 1 || n_ff > nb) return fail(c, PAID_EINVAL, "n_ff must be 1..%d", nb);
  if ((rc = to_host(c, ff, (size_t)n_ff * nb, hff)) != PAID_OK) return rc;
  int identity = 0;
  if ((rc = check_ff(c, hff.data(), n_ff, ff_L, identity)) != PAID_OK) return rc;
  if ((rc = to_host(c, codes, (size_t)n * 3, hc)) != PAID_OK) return rc;
  std::vector<uint64_t> pc(n);
  for (int i = 0; i < n; ++i) {
    int d = hc[3 * i], ix = hc[3 * i + 1], iy = hc[3 * i + 2];
    if (d < 0 || d > 26 || ix < 0 || iy < 0 || ix >= (1 << d) || iy >= (1 << d))
      return fail(c, PAID_EINVAL, "bad rectangle code %d", i);
    pc[i] = make_code(d, (uint64_t)ix, (uint64_t)iy);
  }
  if ((rc = build_tables(c, hp.data(), 1, cfg.kind)) != PAID_OK) return rc;
  HIPCHK(c, c->qv.ensure(sizeof(double) * 2));
  HIPCHK(c, hipMemcpyAsync(c->qv.p, hl.data(), sizeof(double) * 2, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, c->ffc.ensure(sizeof(double) * n_ff * nb));
  HIPCHK(c, hipMemcpyAsync(c->ffc.p, hff.data(), sizeof(double) * n_ff * nb, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, c->ctr.ensure(sizeof(Ctr)));
  HIPCHK(c, launch_container_setup(c->ctr.as<Ctr>(), 1, c->qv.as<double>(), 1, 1,
                                   channel == PAID_PH ? 1 : 0, c->stream));
  const int M = n_ff, MU = M * (M + 1) / 2;
  const long cap = 4L * n;
  DevBuf code, key, Q, si, dv, de, itau, cnt, ctrid, ifl;
  HIPCHK(c, code.ensure(sizeof(uint64_t) * cap));
  HIPCHK(c, key.ensure(sizeof(double) * cap));
  HIPCHK(c, Q.ensure(sizeof(double) * cap * MU));
  HIPCHK(c, si.ensure(sizeof(int) * (8 + (size_t)n)));
  HIPCHK(c, dv.ensure(sizeof(double) * (size_t)n * MU));
  HIPCHK(c, de.ensure(sizeof(double) * (size_t)n));
  HIPCHK(c, itau.ensure(sizeof(float) * MU));
  HIPCHK(c, cnt.ensure(256));
  HIPCHK(c, ifl.ensure(sizeof(int) * (size_t)n));
  HIPCHK(c, hipMemsetAsync(Q.p, 0, sizeof(double) * cap * MU, c->stream));
  HIPCHK(c, hipMemsetAsync(key.p, 0, sizeof(double) * cap, c->stream));
  HIPCHK(c, hipMemcpyAsync(code.p, pc.data(), sizeof(uint64_t) * n, hipMemcpyHostToDevice, c->stream));
  // slot state: cid 0, state active, nleaf n, selcnt n, woff {0, n}, flags, depth; sel = 0..n-1
  std::vector<int> hs(8 + (size_t)n, 0);
  hs[0] = 0;      // cid
  hs[1] = SLOT_ACTIVE;
  hs[2] = n;      // nleaf
  hs[3] = n;      // selcnt
  hs[4] = 0;      // flags
  hs[5] = 0;      // depth
  hs[6] = 0;      // woff[0]
  hs[7] = n;      // woff[1]
  for (int i = 0; i < n; ++i) hs[8 + i] = i;
  HIPCHK(c, hipMemcpyAsync(si.p, hs.data(), sizeof(int) * hs.size(), hipMemcpyHostToDevice, c->stream));
  int hcnt[64] = {0};
  hcnt[4 + 2] = n;  // counters[2]: work items
  HIPCHK(c, hipMemcpyAsync(cnt.p, hcnt, sizeof hcnt, hipMemcpyHostToDevice, c->stream));
  Problem P;
  memset(&P, 0, sizeof P);
  P.entries = c->entries.as<Entry>();
  P.tab = c->tab.as<double>();
  P.tab_rows = c->max_J;
  P.lds_limit = lds_limit(c);
  P.ctr = c->ctr.as<Ctr>();
  P.n_ctr = 1;
  P.kind = cfg.kind;
  P.err_mode = PAID_ERR_GLOBAL;
  P.precision = cfg.precision;
  P.gram = cfg.gram;
  P.gauss_x = cfg.gauss[0];
  P.gauss_y = cfg.gauss[1];
  P.gauss_s = cfg.gauss[2];
  P.L = ff_L;
  P.nb = 2 * ff_L + 1;
  P.MB = nb;
  P.M = M;
  P.MU = MU;
  P.ff_identity = identity;
  P.eval_layout = cfg.eval_layout;
  if (eval_lds_bytes(P) == 0)
    return fail(c, PAID_EINVAL, "frequency-sum table of %d rows does not fit in LDS (T too small against the band)",
                P.tab_rows);
  P.ffc = c->ffc.as<double>();
  P.W = 1;
  P.cap = cap;
  P.bmin = 1;
  P.bmax = n;
  P.code = code.as<uint64_t>();
  P.key = key.as<double>();
  P.Q = Q.as<double>();
  int *s = si.as<int>();
  P.cid = s;
  P.state = s + 1;
  P.nleaf = s + 2;
  P.selcnt = s + 3;
  P.flags = s + 4;
  P.st_depth = s + 5;
  P.woff = s + 6;
  P.sel = s + 8;
  P.itau = itau.as<float>();
  P.dv = dv.as<double>();
  P.de = de.as<double>();
  P.counters = cnt.as<int>() + 4;
  P.ifill = ifl.as<int>();
  HIPCHK(c, launch_eval(P, n < 4096 ? n : 4096, c->stream));
  std::vector<double> hQ((size_t)cap * MU), hk(cap);
  HIPCHK(c, hipMemcpyAsync(hQ.data(), Q.p, sizeof(double) * cap * MU, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(hk.data(), key.p, sizeof(double) * cap, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<double> oq((size_t)n * 4 * MU), oe((size_t)n * 4);
  for (int r = 0; r < n; ++r)
    for (int ch = 0; ch < 4; ++ch) {
      long ri = ch == 0 ? r : n + 3L * r + (ch - 1);
      memcpy(&oq[((size_t)r * 4 + ch) * MU], &hQ[ri * MU], sizeof(double) * MU);
      oe[(size_t)r * 4 + ch] = hk[ri];
    }
  HIPCHK(c, hipMemcpy(q2n, oq.data(), sizeof(double) * oq.size(), hipMemcpyDefault));
  HIPCHK(c, hipMemcpy(err, oe.data(), sizeof(double) * oe.size(), hipMemcpyDefault));
  return PAID_OK;
}


long paid_mlp_nparams(void) { return mlp_layout().total; }

int paid_set_seed_model(paid_ctx *c, const float *w, int dmax, double kappa) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  HIPCHK(c, hipSetDevice(c->cfg.device));
  if (!w) {
    c->seed_on = false;
    return PAID_OK;
  }
  if (dmax < 0 || dmax > 12) return fail(c, PAID_EINVAL, "dmax must be 0..12");
  if (!(kappa > 0) || !std::isfinite(kappa)) return fail(c, PAID_EINVAL, "kappa must be > 0");
  c->seed_dmax = dmax;
  c->seed_kappa = kappa;
  const long np = mlp_layout().total;
  HIPCHK(c, c->seedw.ensure(sizeof(float) * np));
  HIPCHK(c, hipMemcpyAsync(c->seedw.p, w, sizeof(float) * np, hipMemcpyDefault, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<float> chk(np);
  HIPCHK(c, hipMemcpy(chk.data(), c->seedw.p, sizeof(float) * np, hipMemcpyDeviceToHost));
  for (long i = 0; i < np; ++i)
    if (!std::isfinite(chk[i])) {
      c->seed_on = false;
      return fail(c, PAID_EINVAL, "model weight %ld is not finite", i);
    }
  c->seed_on = true;
  return PAID_OK;
}

int paid_set_leaf_output(paid_ctx *c, int *codes, double *q2n, long cap) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  if ((codes == nullptr) != (q2n == nullptr) || (codes && cap < 1))
    return fail(c, PAID_EINVAL, "codes and q2n both or neither, cap >= 1");
  c->leaf_codes = codes;
  c->leaf_q = q2n;
  c->leaf_cap = codes ? cap : 0;
  return PAID_OK;
}

int paid_set_pair_weights(paid_ctx *c, const double *w) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  c->pair_w = w;
  return PAID_OK;
}

int paid_set_label_output(paid_ctx *c, float *features, float *labels) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  c->feat_out = features;
  c->lab_out = labels;
  return PAID_OK;
}

int paid_mlp_forward(paid_ctx *c, const float *w, const float *x, int n, float *y) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  if (!w || !x || !y || n < 0) return fail(c, PAID_EINVAL, "bad arguments");
  if (n == 0) return PAID_OK;
  if (n > (1 << 24)) return fail(c, PAID_EINVAL, "n must be <= 2^24");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  const long np = mlp_layout().total;
  DevBuf tw, tx, ty, act;
  const float *dw, *dx;
  float *dy;
  int rc;
  if ((rc = stage_in(c, w, np, tw, dw)) != PAID_OK) return rc;
  if ((rc = stage_in(c, x, (size_t)n * kMlpIn, tx, dx)) != PAID_OK) return rc;
  if ((rc = stage_out(c, y, (size_t)n * kMlpOut, ty, dy)) != PAID_OK) return rc;
  HIPCHK(c, act.ensure(sizeof(float) * 2 * kMlpHid * (size_t)n));
  MlpAct a;
  memset(&a, 0, sizeof a);
  a.A[0] = act.as<float>();
  a.A[1] = a.A[0] + (size_t)kMlpHid * n;
  a.A[2] = a.A[0];
  HIPCHK(c, mlp_forward(dw, dx, n, a, dy, c->stream));
  if ((rc = finish_out(c, y, dy, (size_t)n * kMlpOut)) != PAID_OK) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PAID_OK;
}

// forward pass, mean squared error and backward pass on device arrays with
// the per-sample buffers of a and the loss in dloss (shared by both entry
// points)
static hipError_t loss_grad_launch(paid_ctx *c, const float *dw, const float *dx, const float *dyl,
                                   int n, MlpAct &a, float *yhat, float *dY, float *dg,
                                   double *dloss) {
  hipError_t e;
  if ((e = mlp_forward(dw, dx, n, a, yhat, c->stream)) != hipSuccess) return e;
  if ((e = mlp_mse(yhat, dyl, (long)n * kMlpOut, dY, dloss, nullptr, c->stream)) != hipSuccess) return e;
  return mlp_backward(dw, dx, n, a, dY, dg, c->stream);
}

int paid_mlp_loss_grad_noalloc(paid_ctx *c, const float *w, const float *x, const float *y, int n,
                               float *grad, double *loss) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  if (!w || !x || !y || !grad || n < 1) return fail(c, PAID_EINVAL, "bad arguments");
  if (n > kNoAllocMaxN)
    return fail(c, PAID_EINVAL, "n = %d exceeds the fixed working memory (at most %d samples)", n,
                kNoAllocMaxN);
  if (!is_device_ptr(w) || !is_device_ptr(x) || !is_device_ptr(y) || !is_device_ptr(grad))
    return fail(c, PAID_EINVAL, "paid_mlp_loss_grad_noalloc takes device arrays only");
  if (!c->noalloc) return fail(c, PAID_EINTERNAL, "fixed working memory not set up");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  // carve the per-sample buffers of n samples and the loss from the array
  const size_t h = (size_t)kMlpHid * n, o = (size_t)kMlpOut * n;
  float *p = c->noalloc;
  MlpAct a;
  for (int l = 0; l < 3; ++l) {
    a.Z[l] = p + (size_t)l * h;
    a.A[l] = p + (size_t)(3 + l) * h;
    a.D[l] = p + (size_t)(6 + l) * h;
  }
  a.Z[3] = nullptr;
  float *yhat = p + 9 * h, *dY = yhat + o;
  double *dloss = reinterpret_cast<double *>(p + kNoAllocActFloats);
  HIPCHK(c, loss_grad_launch(c, w, x, y, n, a, yhat, dY, grad, dloss));
  // the loss goes through the context's pinned buffer (bytes 32..39)
  double *hl = reinterpret_cast<double *>(reinterpret_cast<char *>(c->host_counters) + 32);
  HIPCHK(c, hipMemcpyAsync(hl, dloss, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (loss) *loss = *hl;
  return PAID_OK;
}

int paid_mlp_loss_grad(paid_ctx *c, const float *w, const float *x, const float *y, int n,
                       float *grad, double *loss) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  if (!w || !x || !y || !grad || n < 1 || n > 65536) return fail(c, PAID_EINVAL, "bad arguments");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  const long np = mlp_layout().total;
  DevBuf tw, tx, ty, tg, act, tl;
  const float *dw, *dx, *dyl;
  float *dg;
  int rc;
  if ((rc = stage_in(c, w, np, tw, dw)) != PAID_OK) return rc;
  if ((rc = stage_in(c, x, (size_t)n * kMlpIn, tx, dx)) != PAID_OK) return rc;
  if ((rc = stage_in(c, y, (size_t)n * kMlpOut, ty, dyl)) != PAID_OK) return rc;
  if ((rc = stage_out(c, grad, np, tg, dg)) != PAID_OK) return rc;
  MlpAct a;
  float *yhat, *dY;
  if ((rc = carve_act(c, act, n, a, yhat, dY)) != PAID_OK) return rc;
  HIPCHK(c, tl.ensure(sizeof(double)));
  HIPCHK(c, loss_grad_launch(c, dw, dx, dyl, n, a, yhat, dY, dg, tl.as<double>()));
  if ((rc = finish_out(c, grad, dg, np)) != PAID_OK) return rc;
  double hl = 0.0;
  HIPCHK(c, hipMemcpyAsync(&hl, tl.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (loss) *loss = hl;
  return PAID_OK;
}

int paid_mlp_adam(paid_ctx *c, float *w, const float *g, float *m, float *v, int t, float lr) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  if (!w || !g || !m || !v || t < 1 || !(lr > 0)) return fail(c, PAID_EINVAL, "bad arguments");
  if (!is_device_ptr(w) || !is_device_ptr(g) || !is_device_ptr(m) || !is_device_ptr(v))
    return fail(c, PAID_EINVAL, "paid_mlp_adam needs device arrays");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  HIPCHK(c, mlp_adam(w, g, m, v, mlp_layout().total, t, nullptr, lr, lr, 0, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PAID_OK;
}

int paid_train_opts_default(paid_train_opts *o) {
  if (!o) return PAID_EINVAL;
  memset(o, 0, sizeof *o);
  o->steps = 3000;
  o->batch = 256;
  o->lr = 2e-3f;
  o->lr_final = 5e-5f;
  o->seed = 1;
  o->init = 1;
  o->use_graph = 1;
  return PAID_OK;
}

int paid_seed_train(paid_ctx *c, const float *x, const float *y, int n, const paid_train_opts *oin,
                    float *w, double *loss_hist) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  paid_train_opts o;
  if (oin) o = *oin; else paid_train_opts_default(&o);
  if (!x || !y || !w || n < 1) return fail(c, PAID_EINVAL, "bad arguments");
  if (o.steps < 1 || o.batch < 1 || o.batch > 1024 || !(o.lr > 0) || !(o.lr_final >= 0))
    return fail(c, PAID_EINVAL, "bad training options");
  if ((long)o.steps * o.batch > (1L << 30)) return fail(c, PAID_EINVAL, "steps * batch too large");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  const MlpLayout L = mlp_layout();
  const long np = L.total;
  const int bs = o.batch;
  DevBuf tx, ty, wd, mv, idx, ctr, hist, xb, act, gr;
  const float *dx, *dy;
  int rc;
  if ((rc = stage_in(c, x, (size_t)n * kMlpIn, tx, dx)) != PAID_OK) return rc;
  if ((rc = stage_in(c, y, (size_t)n * kMlpOut, ty, dy)) != PAID_OK) return rc;
  HIPCHK(c, wd.ensure(sizeof(float) * np));
  if (o.init) {
    std::mt19937_64 gen(o.seed ^ 0x5eed5eedULL);
    std::vector<float> hw(np, 0.0f);
    for (int l = 0; l < 4; ++l) {
      std::normal_distribution<double> nd(0.0, 1.0 / sqrt((double)L.ni[l]));
      for (long k = 0; k < (long)L.no[l] * L.ni[l]; ++k) hw[L.w[l] + k] = (float)nd(gen);
    }
    HIPCHK(c, hipMemcpyAsync(wd.p, hw.data(), sizeof(float) * np, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    HIPCHK(c, hipMemcpyAsync(wd.p, w, sizeof(float) * np, hipMemcpyDefault, c->stream));
  }
  HIPCHK(c, mv.ensure(sizeof(float) * 2 * np));
  HIPCHK(c, hipMemsetAsync(mv.p, 0, sizeof(float) * 2 * np, c->stream));
  // minibatch indices: consecutive passes over shuffled orders of the samples
  {
    std::mt19937_64 gen(o.seed);
    std::vector<int> perm(n), hidx((size_t)o.steps * bs);
    for (int i = 0; i < n; ++i) perm[i] = i;
    size_t k = 0;
    while (k < hidx.size()) {
      for (int i = n - 1; i > 0; --i) {
        std::uniform_int_distribution<int> ud(0, i);
        std::swap(perm[i], perm[ud(gen)]);
      }
      for (int i = 0; i < n && k < hidx.size(); ++i) hidx[k++] = perm[i];
    }
    HIPCHK(c, idx.ensure(sizeof(int) * hidx.size()));
    HIPCHK(c, hipMemcpyAsync(idx.p, hidx.data(), sizeof(int) * hidx.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  HIPCHK(c, ctr.ensure(sizeof(int)));
  HIPCHK(c, hipMemsetAsync(ctr.p, 0, sizeof(int), c->stream));
  HIPCHK(c, hist.ensure(sizeof(double) * o.steps));
  HIPCHK(c, xb.ensure(sizeof(float) * (size_t)bs * (kMlpIn + kMlpOut)));
  HIPCHK(c, gr.ensure(sizeof(float) * np));
  MlpAct a;
  float *yhat, *dY;
  if ((rc = carve_act(c, act, bs, a, yhat, dY)) != PAID_OK) return rc;
  float *Xb = xb.as<float>(), *Yb = Xb + (size_t)bs * kMlpIn;
  float *W = wd.as<float>(), *M = mv.as<float>(), *V = M + np, *G = gr.as<float>();
  int *step = ctr.as<int>();
  double *lh = hist.as<double>();
  auto one_step = [&](hipStream_t st) -> hipError_t {
    hipError_t e;
    if ((e = mlp_gather(dx, dy, idx.as<int>(), step, bs, Xb, Yb, st)) != hipSuccess) return e;
    if ((e = mlp_forward(W, Xb, bs, a, yhat, st)) != hipSuccess) return e;
    if ((e = mlp_mse(yhat, Yb, (long)bs * kMlpOut, dY, lh, step, st)) != hipSuccess) return e;
    if ((e = mlp_backward(W, Xb, bs, a, dY, G, st)) != hipSuccess) return e;
    if ((e = mlp_adam(W, G, M, V, np, 0, step, o.lr, o.lr_final, o.steps, st)) != hipSuccess) return e;
    return mlp_count(step, st);
  };
  if (o.use_graph) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    hipError_t e = one_step(c->stream);
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      HIPCHK(c, e != hipSuccess ? e : e2);
    }
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(c, e);
    for (int t = 0; t < o.steps && e == hipSuccess; ++t) e = hipGraphLaunch(ge, c->stream);
    hipError_t e3 = hipStreamSynchronize(c->stream);
    (void)hipGraphExecDestroy(ge);
    HIPCHK(c, e);
    HIPCHK(c, e3);
  } else {
    for (int t = 0; t < o.steps; ++t) HIPCHK(c, one_step(c->stream));
  }
  HIPCHK(c, hipMemcpyAsync(w, W, sizeof(float) * np, hipMemcpyDefault, c->stream));
  if (loss_hist)
    HIPCHK(c, hipMemcpyAsync(loss_hist, lh, sizeof(double) * o.steps, hipMemcpyDefault, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PAID_OK;
}

int paid_contract(paid_ctx *c, int n_l, int M, const double *chi, const double *VP,
                  const double *VC, const double *VD, double *dP, double *dC, double *dD) {
  if (!c) return PAID_EINVAL;
  c->err.clear();
  if (n_l < 0 || M < 1 || M > 32) return fail(c, PAID_EINVAL, "need n_l >= 0 and 1 <= M <= 32");
  if (n_l == 0) return PAID_OK;
  if (!chi || !VP || !VC || !VD || !dP || !dC || !dD) return fail(c, PAID_EINVAL, "NULL array");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  const size_t n = (size_t)n_l * M * M;
  DevBuf tc, tp, tcc, td, o1, o2, o3;
  const double *dchi, *dvp, *dvc, *dvd;
  double *rp, *rc, *rd;
  int rc_;
  if ((rc_ = stage_in(c, chi, 2 * n, tc, dchi)) != PAID_OK) return rc_;
  if ((rc_ = stage_in(c, VP, n, tp, dvp)) != PAID_OK) return rc_;
  if ((rc_ = stage_in(c, VC, n, tcc, dvc)) != PAID_OK) return rc_;
  if ((rc_ = stage_in(c, VD, n, td, dvd)) != PAID_OK) return rc_;
  if ((rc_ = stage_out(c, dP, n, o1, rp)) != PAID_OK) return rc_;
  if ((rc_ = stage_out(c, dC, n, o2, rc)) != PAID_OK) return rc_;
  if ((rc_ = stage_out(c, dD, n, o3, rd)) != PAID_OK) return rc_;
  HIPCHK(c, launch_contract(n_l, M, dchi, dvp, dvc, dvd, rp, rc, rd, c->stream));
  if ((rc_ = finish_out(c, dP, rp, n)) != PAID_OK) return rc_;
  if ((rc_ = finish_out(c, dC, rc, n)) != PAID_OK) return rc_;
  if ((rc_ = finish_out(c, dD, rd, n)) != PAID_OK) return rc_;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PAID_OK;
}

int paid_flow_opts_default(paid_flow_opts *o) {
  if (!o) return PAID_EINVAL;
  memset(o, 0, sizeof *o);
  o->omega0 = 1.0;
  o->omega1 = 0.1;
  o->rtol = 1e-6;
  o->atol = 0.0;
  o->rtol_int = 1e-8;
  o->h0 = 0.0;
  o->max_steps = 200;
  return PAID_OK;
}

int paid_flow(paid_ctx *c, const paid_params *base, const double *q, int n_q, const double *ff,
              int n_ff, int ff_L, const double *VP, const double *VC, const double *VD, double *P,
              double *C, double *D, const paid_flow_opts *oin, paid_flow_stats *stats) {
  auto t0 = std::chrono::steady_clock::now();
  if (!c) return PAID_EINVAL;
  c->err.clear();
  paid_flow_opts o;
  if (oin) o = *oin; else paid_flow_opts_default(&o);
  if (!base || !q || !ff || !VP || !VC || !VD || !P || !C || !D || n_q < 1 || n_ff < 1 || n_ff > 32)
    return fail(c, PAID_EINVAL, "bad arguments");
  if (!(o.omega0 > 0) || !(o.omega1 > 0) || !(o.rtol >= 0) || !(o.atol >= 0) ||
      !(o.rtol > 0 || o.atol > 0) || !(o.rtol_int > 0) || o.max_steps < 1)
    return fail(c, PAID_EINVAL, "bad flow options");
  if (c->cfg.kind != PAID_BUBBLE_DOT) return fail(c, PAID_EINVAL, "the flow needs kind PAID_BUBBLE_DOT");
  for (const void *a : {(const void *)VP, (const void *)VC, (const void *)VD, (const void *)P,
                        (const void *)C, (const void *)D})
    if (is_device_ptr(a)) return fail(c, PAID_EINVAL, "the flow takes couplings and state in host memory");
  const int M = n_ff;
  const size_t nm = (size_t)n_q * M * M, ny = 3 * nm;  // state: P, C, D
  std::vector<double> y(ny), V(ny);
  memcpy(y.data(), P, sizeof(double) * nm);
  memcpy(y.data() + nm, C, sizeof(double) * nm);
  memcpy(y.data() + 2 * nm, D, sizeof(double) * nm);
  memcpy(V.data(), VP, sizeof(double) * nm);
  memcpy(V.data() + nm, VC, sizeof(double) * nm);
  memcpy(V.data() + 2 * nm, VD, sizeof(double) * nm);
  std::vector<double> chi(2 * nm), rhs(ny);
  paid_flow_stats st;
  memset(&st, 0, sizeof st);
  // f(s) = dy/d(ln Omega) = Omega dy/dOmega at Omega = e^s (independent of y)
  auto f = [&](double s, double *out) -> int {
    paid_params p = *base;
    p.Omega = exp(s);
    paid_stats is;
    int rc = paid_integrate(c, &p, 1, q, n_q, ff, n_ff, ff_L, PAID_PP | PAID_PH, o.rtol_int, 0.0,
                            chi.data(), nullptr, &is);
    if (rc == PAID_ENOCONV)
      return fail(c, PAID_ENOCONV, "flow: the integration at Omega = %g hit max_regions", p.Omega);
    if (rc != PAID_OK) return rc;
    st.evaluations++;
    st.kernel_evals += is.kernel_evals;
    rc = paid_contract(c, n_q, M, chi.data(), V.data(), V.data() + nm, V.data() + 2 * nm, out,
                       out + nm, out + 2 * nm);
    if (rc != PAID_OK) return rc;
    for (size_t i = 0; i < ny; ++i) out[i] *= p.Omega;
    return PAID_OK;
  };
  // Dormand-Prince 5(4): nodes, stage weights, 5th-order and 4th-order weights
  static const double cc[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
  static const double b5[7] = {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0.0};
  static const double b4[7] = {5179.0 / 57600, 0.0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200,
                               187.0 / 2100, 1.0 / 40};
  const double s0 = log(o.omega0), s1 = log(o.omega1), dir = s1 >= s0 ? 1.0 : -1.0;
  double s = s0;
  double h = o.h0 > 0 ? dir * o.h0 : 0.1 * (s1 - s0);
  if (h == 0.0) {
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return PAID_OK;
  }
  std::vector<std::vector<double>> k(7, std::vector<double>(ny));
  int rc = f(s, k[0].data());
  if (rc != PAID_OK) return rc;
  while (dir * (s1 - s) > 1e-14 * fabs(s1 - s0)) {
    if (st.steps + st.rejected >= o.max_steps)
      return fail(c, PAID_ENOCONV, "flow: %d steps without reaching omega1", o.max_steps);
    if (dir * (s + h - s1) > 0) h = s1 - s;
    // the right-hand side does not depend on the state: stages are f(s + c h)
    for (int i = 1; i < 7; ++i)
      if ((rc = f(s + cc[i] * h, k[i].data())) != PAID_OK) return rc;
    double emax = 0.0, ymax = 0.0;
    std::vector<double> yn(ny);
    for (size_t j = 0; j < ny; ++j) {
      double d5 = 0.0, d4 = 0.0;
      for (int i = 0; i < 7; ++i) {
        d5 += b5[i] * k[i][j];
        d4 += b4[i] * k[i][j];
      }
      yn[j] = y[j] + h * d5;
      emax = fmax(emax, fabs(h * (d5 - d4)));
      ymax = fmax(ymax, fmax(fabs(y[j]), fabs(yn[j])));
    }
    const double tol = o.atol + o.rtol * ymax;
    const double ratio = tol > 0 ? emax / tol : (emax > 0 ? 1e300 : 0.0);
    if (ratio <= 1.0) {
      y.swap(yn);
      s += h;
      st.steps++;
      k[0].swap(k[6]);  // first same as last
    } else {
      st.rejected++;
    }
    const double fac = ratio > 0 ? 0.9 * pow(ratio, -0.2) : 5.0;
    h *= fmin(5.0, fmax(0.2, fac));
  }
  memcpy(P, y.data(), sizeof(double) * nm);
  memcpy(C, y.data() + nm, sizeof(double) * nm);
  memcpy(D, y.data() + 2 * nm, sizeof(double) * nm);
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  return PAID_OK;
}

}  // extern "C"
