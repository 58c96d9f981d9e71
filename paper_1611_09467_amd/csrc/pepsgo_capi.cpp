// Host side of the C-ABI: argument checks, shape planning, workspace layout and
// the launch sequence of one evaluation (see include/pepsgo.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pepsgo.h"
#include "pepsgo_internal.h"
#include "pg_device.h"

using namespace pg;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(PEPSGO_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

}  // namespace

namespace pg {

int api_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace pg

struct pepsgo_ctx_ {
  int device;
  int lds_budget;  // bytes of LDS a workgroup may use
  void* scratch = nullptr;  // device address of the fixed workspace on this device
  int profiling = 0;
  std::mutex prof_mu;  // guards recs/pool/totals: evaluations may come from several threads
  // LDS budgets chosen per (D, Dc, precision), by pepsgo_autotune or pepsgo_tune_set
  std::mutex tune_mu;
  std::map<std::tuple<int, int, int>, pepsgo_tuning> tune;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;         // events recorded since the last read/reset
  std::vector<hipEvent_t> pool;  // reusable events
  double total_ms[PEPSGO_K_COUNT] = {0};
  int64_t launches[PEPSGO_K_COUNT] = {0};
};

struct pepsgo_graph_ {
  int device;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

struct pepsgo_peps_ {
  pepsgo_ctx ctx;
  int N, M, d, D;
  int64_t nparams;
  double* dT;
  int64_t* d_site_off;
  int64_t* d_grad_off;
  double* d_ones;
  std::vector<int64_t> site_off, grad_off;
  int64_t grad_elems;
};

namespace {

struct Plan {
  int N, M, D, Dc, chimax;
  int64_t site_slot, env_stride, re_slot, re2_slot;
  int n_env;
  int64_t off_envlog, off_rowlog, off_rowsign, off_eloc, off_flags, off_re, off_re2, off_grad,
      off_scratch;
  int64_t ws_stride;  // doubles
  BufPlan zip, sand, strip, strip64;  // strip64: float64 re-run of rejected reduced-precision strips
  int lds_zip, lds_sand, lds_strip, lds_strip64;
  int xc, xc64;                       // x values per stage of the strip update (strip, strip64)
  int eig_batch;
  int lw_doubles;
  int c_doubles;
  int zip_threads;  // 64: one wave per sample; 256: four waves
};

// Assign buffers (sizes in doubles) to LDS in order while they fit; the rest
// go to the sample's global scratch.  Returns the global scratch size.
int64_t place(const std::vector<int64_t>& sizes, int budget_bytes, BufPlan* bp, int* lds_bytes) {
  int64_t lds = 0, glob = 0;
  bp->glob = 0;
  for (size_t b = 0; b < sizes.size(); ++b) {
    const int64_t n = round_up(sizes[b], 4);
    if ((lds + n) * 8 <= budget_bytes) {
      bp->off[b] = lds;
      lds += n;
    } else {
      bp->off[b] = glob;
      glob += n;
      bp->glob |= 1u << b;
    }
  }
  *lds_bytes = (int)(lds * 8);
  return glob;
}

// LDS budgets used when nothing was tuned for a shape: the truncation and
// strip kernels keep two workgroups per CU (80 KB each) in float64, the strip
// four (40 KB) with float32 storage; the sandwich takes what it needs.
pepsgo_tuning default_tuning(int precision, int lds_budget) {
  pepsgo_tuning t;
  t.zip_lds_bytes = 0;  // by shape: one-wave workgroups (20 KB) where blocks fit, else 80 KB
  t.sandwich_lds_bytes = lds_budget;
  t.strip_lds_bytes = std::min(lds_budget, precision == PEPSGO_FP64 ? 80 * 1024 : 40 * 1024);
  t.strip_xc = 1;
  return t;
}

pepsgo_tuning tuning_for(pepsgo_ctx_* c, int D, int Dc, int precision) {
  std::lock_guard<std::mutex> g(c->tune_mu);
  auto it = c->tune.find(std::make_tuple(D, Dc, precision));
  return it != c->tune.end() ? it->second : default_tuning(precision, c->lds_budget);
}

Plan make_plan(const pepsgo_peps_* P, int Dc, int want_eloc, int precision, const pepsgo_tuning& tn,
               int grad_mode = PEPSGO_GRAD_NONE) {
  Plan p;
  p.N = P->N;
  p.M = P->M;
  p.D = P->D;
  p.Dc = Dc;
  const int64_t chi = std::max(Dc, P->D), D = P->D;
  p.chimax = (int)chi;
  p.site_slot = round_up(chi * D * chi, 4);
  p.env_stride = p.site_slot * p.M;
  p.re_slot = round_up(chi * D * chi, 4);
  p.re2_slot = want_eloc ? round_up(chi * D * D * chi, 4) : 0;
  p.n_env = p.N + 2;
  int64_t o = (int64_t)p.n_env * p.env_stride;
  p.off_envlog = o;
  o += round_up(p.n_env, 4);
  p.off_rowlog = o;
  o += round_up(p.N, 4);
  p.off_rowsign = o;
  o += round_up(p.N, 4);
  p.off_eloc = o;
  o += 4;
  p.off_flags = o;
  o += 4;
  p.off_re = o;
  o += (p.M + 1) * p.re_slot;
  p.off_re2 = o;
  o += (p.M + 1) * p.re2_slot;
  // REDUCED gradients: each sample's Delta block stays in its workspace until
  // the chunk's Eq. (3) sums are taken
  p.off_grad = o;
  if (grad_mode == PEPSGO_GRAD_REDUCED) o += round_up(P->grad_elems, 4);
  p.off_scratch = o;

  const int budget = P->ctx->lds_budget;
  auto clampb = [&](int b) { return std::max(1024, std::min(budget, b)); };
  const int64_t red = kRedDoubles + 2 * (kMaxSide + 1);
  const int64_t rowsmax = chi * D;
  // truncation kernel.  Blocks up to 72 x 72: one wave per sample by default
  // (or when the budget asked for is at most 40 KB), eight per CU at 20 KB of
  // LDS: work arrays and vectors in LDS, the rest in the sample's scratch.
  // Otherwise four waves per sample, two workgroups per CU at 80 KB.
  const bool wave = rowsmax <= 72 && tn.zip_lds_bytes <= 40 * 1024;
  p.zip_threads = wave ? 64 : 256;
  std::vector<int64_t> zs(ZB_COUNT);
  zs[ZB_RED] = 64;
  zs[ZB_MISC] = 4 * chi + 8;
  zs[ZB_G] = std::max({rowsmax * rowsmax, chi * D * D * chi, chi * D * chi});
  // eigensolver work followed by the eigenvectors; also the LQ reflectors and a staged MPS tensor
  zs[ZB_V] = std::max<int64_t>(top_svd_work((int)rowsmax, (int)rowsmax, (int)chi, wave) + rowsmax * chi,
                               chi * D * chi);
  zs[ZB_C] = std::max(chi * chi * D, 2 * chi * chi);
  zs[ZB_X] = std::max(rowsmax * rowsmax, chi * D * chi);
  // LQ output and staged slices; one inverse iteration (8 rowsmax) plus the
  // Gram-Schmidt coefficients; the Cholesky-QR factor; the Sturm counts
  const int64_t lw_min = std::max({chi * D * chi, D * D * D * D, 8 * rowsmax + chi,
                                   chi * chi + 2 * chi + 1, (int64_t)2 * kZipThreads});
  auto round4 = [](int64_t v) { return round_up(v, 4); };
  const int64_t fixed = round4(zs[ZB_RED]) + round4(zs[ZB_MISC]) + round4(zs[ZB_G]) +
                        round4(zs[ZB_V]) + round4(zs[ZB_C]);
  int zbudget;
  int64_t lw;
  std::vector<int> zorder;
  if (wave) {
    zbudget = clampb(tn.zip_lds_bytes ? tn.zip_lds_bytes : 20 * 1024);
    lw = std::max(lw_min, 8 * rowsmax * chi + chi);  // in the scratch: every vector at once
    zorder = {ZB_RED, ZB_MISC, ZB_V, ZB_C, ZB_LW, ZB_X, ZB_G};
  } else {
    zbudget = clampb(tn.zip_lds_bytes ? tn.zip_lds_bytes : 80 * 1024);
    if ((fixed + round4(lw_min)) * 8 > zbudget) zbudget = budget;
    lw = std::max(lw_min, std::min<int64_t>(8 * rowsmax * chi + chi, zbudget / 8 - fixed - 4));
    zorder = {ZB_RED, ZB_MISC, ZB_G, ZB_V, ZB_C, ZB_LW, ZB_X};
  }
  p.eig_batch = (int)std::max<int64_t>(1, std::min<int64_t>(chi, (lw - chi) / (8 * rowsmax)));
  p.lw_doubles = (int)lw;
  p.c_doubles = (int)zs[ZB_C];
  zs[ZB_LW] = lw;
  {
    std::vector<int64_t> sz;
    for (int b : zorder) sz.push_back(zs[b]);
    BufPlan tmp;
    int64_t g = place(sz, zbudget, &tmp, &p.lds_zip);
    p.zip.glob = 0;
    for (size_t q = 0; q < zorder.size(); ++q) {
      p.zip.off[zorder[q]] = tmp.off[q];
      if ((tmp.glob >> q) & 1u) p.zip.glob |= 1u << zorder[q];
    }
    p.ws_stride = g;  // temporarily the scratch need
  }
  std::vector<int64_t> ss(SB_COUNT);
  ss[SB_RED] = red;
  ss[SB_T1] = D * chi * D * chi;
  ss[SB_T2] = chi * chi * D * D;
  ss[SB_LE0] = chi * D * chi;
  ss[SB_LE1] = chi * D * chi;
  ss[SB_E1] = chi * D * chi;
  ss[SB_E2] = chi * D * chi;
  ss[SB_Q] = chi * chi * D * D;
  ss[SB_STG] = D * D * D * D + chi * D * chi;
  std::vector<int> sorder = {SB_RED, SB_STG, SB_T1, SB_T2, SB_LE0, SB_LE1, SB_E1, SB_E2, SB_Q};
  int64_t gs;
  {
    std::vector<int64_t> sz;
    for (int b : sorder) sz.push_back(ss[b]);
    BufPlan tmp;
    gs = place(sz, clampb(tn.sandwich_lds_bytes), &tmp, &p.lds_sand);
    p.sand.glob = 0;
    for (size_t q = 0; q < sorder.size(); ++q) {
      p.sand.off[sorder[q]] = tmp.off[q];
      if ((tmp.glob >> q) & 1u) p.sand.glob |= 1u << sorder[q];
    }
  }
  // strip buffers hold float64 or float32 elements (sizes below in elements)
  auto strip_sizes = [&](int64_t es, int64_t xc) {
    auto in_doubles = [&](int64_t n) { return (n * es + 7) / 8; };
    std::vector<int64_t> ts(TB_COUNT);
    ts[TB_RED] = red;
    // odd leading dimensions of the strip intermediates; xc slots of each
    const int64_t ld1 = (D * D) | 1, ld3 = (chi * D) | 1;
    ts[TB_T1] = in_doubles(xc * std::max(D * chi * ld1, D * D * ld3));  // also holds the third intermediate
    ts[TB_T2] = in_doubles(xc * chi * D * ld1);
    ts[TB_STG] = in_doubles(2 * chi * D * chi + 2 * D * D * D * D);
    ts[TB_LE0] = in_doubles(chi * D * D * chi);
    ts[TB_LE1] = in_doubles(chi * D * D * chi);
    ts[TB_E1] = in_doubles(chi * D * D * chi);
    ts[TB_E2] = in_doubles(chi * D * D * chi);
    return ts;
  };
  int64_t gt = 0;
  p.lds_strip = p.lds_strip64 = 0;
  p.xc = std::max(1, std::min(4, tn.strip_xc));
  const pepsgo_tuning t64 = tuning_for(P->ctx, P->D, Dc, PEPSGO_FP64);
  p.xc64 = std::max(1, std::min(4, t64.strip_xc));
  if (want_eloc) {
    gt = place(strip_sizes(precision == PEPSGO_FP64 ? 8 : 4, p.xc), clampb(tn.strip_lds_bytes),
               &p.strip, &p.lds_strip);
    gt = std::max(gt, place(strip_sizes(8, p.xc64), clampb(t64.strip_lds_bytes), &p.strip64,
                            &p.lds_strip64));
  }
  const int64_t scratch = std::max({p.ws_stride, gs, gt});
  p.ws_stride = round_up(p.off_scratch + scratch, 32);
  return p;
}

void row_bonds(int M, int D, int* out) {
  out[0] = 1;
  for (int j = 1; j < M; ++j) out[j] = D;
  out[M] = 1;
}

ZipShape make_zip(const Plan& p, const int* chi_in, int row, int dir) {
  ZipShape z;
  std::memset(&z, 0, sizeof z);
  z.row = row;
  z.dir = dir;
  const int M = p.M;
  std::vector<int> pin(M), pout(M), dr(M);
  for (int j = 0; j < M; ++j) {
    int a, b, c, d;
    site_dims(p.N, p.M, p.D, row, j, &a, &b, &c, &d);
    pin[j] = dir == 0 ? c : d;
    pout[j] = dir == 0 ? d : c;
    dr[j] = b;
  }
  for (int j = 0; j <= M; ++j) z.chi_in[j] = chi_in[j];
  z.chic[M] = 1;
  for (int j = M - 1; j >= 1; --j) z.chic[j] = std::min(chi_in[j], pin[j] * z.chic[j + 1]);
  z.chic[0] = 1;
  z.nb[0] = 1;
  for (int j = 0; j < M - 1; ++j) {
    const int rows = z.nb[j] * pout[j], cols = z.chic[j + 1] * dr[j];
    z.nb[j + 1] = std::min({p.Dc, rows, cols});
  }
  z.nb[M] = 1;
  z.eig_batch = p.eig_batch;
  z.lw_doubles = p.lw_doubles;
  z.c_doubles = p.c_doubles;
  z.threads = p.zip_threads;
  return z;
}

// Bracket one launch with events when profiling is on.
struct Timed {
  pepsgo_ctx_* c;
  int cls;
  hipStream_t s;
  hipEvent_t a{}, b{};
  bool on = false;
  Timed(pepsgo_ctx_* c_, int cls_, hipStream_t s_, bool allowed = true) : c(c_), cls(cls_), s(s_) {
    if (!allowed || !c->profiling) return;
    std::lock_guard<std::mutex> g(c->prof_mu);
    on = true;
    a = take();
    b = take();
    (void)hipEventRecord(a, s);
  }
  hipEvent_t take() {
    if (!c->pool.empty()) {
      hipEvent_t e = c->pool.back();
      c->pool.pop_back();
      return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
  ~Timed() {
    if (!on) return;
    std::lock_guard<std::mutex> g(c->prof_mu);
    (void)hipEventRecord(b, s);
    c->recs.push_back({cls, a, b});
  }
};

void drain_profile(pepsgo_ctx_* c) {
  std::lock_guard<std::mutex> g(c->prof_mu);
  for (auto& r : c->recs) {
    (void)hipEventSynchronize(r.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->total_ms[r.cls] += ms;
      c->launches[r.cls] += 1;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
}

}  // namespace

extern "C" {

int pepsgo_profile(pepsgo_ctx ctx, int enable) {
  if (!ctx) return fail(PEPSGO_EINVAL, "pepsgo_profile: NULL context");
  if (enable < 0) {
    drain_profile(ctx);
    std::lock_guard<std::mutex> g(ctx->prof_mu);
    for (int k = 0; k < PEPSGO_K_COUNT; ++k) {
      ctx->total_ms[k] = 0.0;
      ctx->launches[k] = 0;
    }
    return PEPSGO_OK;
  }
  ctx->profiling = enable ? 1 : 0;
  return PEPSGO_OK;
}

int pepsgo_profile_read(pepsgo_ctx ctx, int cls, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return fail(PEPSGO_EINVAL, "pepsgo_profile_read: NULL argument");
  if (cls < 0 || cls >= PEPSGO_K_COUNT) return fail(PEPSGO_EINVAL, "pepsgo_profile_read: class %d", cls);
  drain_profile(ctx);
  std::lock_guard<std::mutex> g(ctx->prof_mu);
  *total_ms = ctx->total_ms[cls];
  *launches = ctx->launches[cls];
  return PEPSGO_OK;
}

int pepsgo_version(int* major, int* minor) {
  if (major) *major = PEPSGO_VERSION_MAJOR;
  if (minor) *minor = PEPSGO_VERSION_MINOR;
  return PEPSGO_OK;
}

const char* pepsgo_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace pg {
int ctx_device(pepsgo_ctx c) { return c->device; }
void peps_shape(pepsgo_peps p, int* N, int* M) {
  *N = p->N;
  *M = p->M;
}
}  // namespace pg

extern "C" {

int pepsgo_create(int hip_device, pepsgo_ctx* out) {
  if (!out) return fail(PEPSGO_EINVAL, "pepsgo_create: out is NULL");
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n)
    return fail(PEPSGO_EINVAL, "pepsgo_create: device %d out of range (%d devices)", hip_device, n);
  HIP_TRY(hipSetDevice(hip_device));
  int lds = 0;
  HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device));
  // the fixed workspace of pepsgo_evaluate_noalloc: its address on this device
  void* scr = nullptr;
  HIP_TRY(scratch_address(&scr));
  if (!scr) return fail(PEPSGO_EDEVICE, "pepsgo_create: no device address for the fixed workspace");
  auto* c = new pepsgo_ctx_;
  c->device = hip_device;
  c->lds_budget = std::min(lds, 160 * 1024);
  c->scratch = scr;
  *out = c;
  return PEPSGO_OK;
}

int pepsgo_destroy(pepsgo_ctx ctx) {
  if (!ctx) return fail(PEPSGO_EINVAL, "pepsgo_destroy: NULL context");
  drain_profile(ctx);
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  delete ctx;
  return PEPSGO_OK;
}

int pepsgo_peps_load(pepsgo_ctx ctx, int nrows, int ncols, int d, int D, const double* tensors,
                     int on_device, pepsgo_peps* out) {
  if (!ctx || !out || !tensors) return fail(PEPSGO_EINVAL, "pepsgo_peps_load: NULL argument");
  if (d != 2) return fail(PEPSGO_EUNSUPPORTED, "pepsgo_peps_load: physical dimension %d (only 2)", d);
  if (nrows < 2 || ncols < 2 || D < 1)
    return fail(PEPSGO_EINVAL, "pepsgo_peps_load: need nrows, ncols >= 2 and D >= 1 (got %d, %d, %d)",
                nrows, ncols, D);
  if (nrows > PEPSGO_MAX_SIDE || ncols > PEPSGO_MAX_SIDE || D > PEPSGO_MAX_D)
    return fail(PEPSGO_EUNSUPPORTED, "pepsgo_peps_load: %dx%d D=%d beyond the limits (%d, %d)", nrows,
                ncols, D, PEPSGO_MAX_SIDE, PEPSGO_MAX_D);
  HIP_TRY(hipSetDevice(ctx->device));
  auto* P = new pepsgo_peps_;
  P->ctx = ctx;
  P->N = nrows;
  P->M = ncols;
  P->d = d;
  P->D = D;
  int64_t off = 0, goff = 0;
  for (int i = 0; i < nrows; ++i)
    for (int j = 0; j < ncols; ++j) {
      int a, b, c, e;
      site_dims(nrows, ncols, D, i, j, &a, &b, &c, &e);
      P->site_off.push_back(off);
      P->grad_off.push_back(goff);
      off += (int64_t)d * a * b * c * e;
      goff += (int64_t)a * b * c * e;
    }
  P->nparams = off;
  P->grad_elems = goff;
  P->dT = nullptr;
  P->d_site_off = P->d_grad_off = nullptr;
  P->d_ones = nullptr;
  auto cleanup = [&](int code, const char* what) {
    (void)hipFree(P->dT);
    (void)hipFree(P->d_site_off);
    (void)hipFree(P->d_grad_off);
    (void)hipFree(P->d_ones);
    delete P;
    return fail(code, "pepsgo_peps_load: %s", what);
  };
  if (hipMalloc(&P->dT, off * sizeof(double)) != hipSuccess) return cleanup(PEPSGO_ENOMEM, "tensor allocation");
  if (hipMalloc(&P->d_site_off, P->site_off.size() * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&P->d_grad_off, P->grad_off.size() * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&P->d_ones, 64 * sizeof(double)) != hipSuccess)
    return cleanup(PEPSGO_ENOMEM, "index allocation");
  std::vector<double> ones(64, 1.0);
  if (hipMemcpy(P->dT, tensors, off * sizeof(double),
                on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->d_site_off, P->site_off.data(), P->site_off.size() * sizeof(int64_t),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->d_grad_off, P->grad_off.data(), P->grad_off.size() * sizeof(int64_t),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->d_ones, ones.data(), 64 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(PEPSGO_EDEVICE, "copy to device");
  *out = P;
  return PEPSGO_OK;
}

int pepsgo_peps_update(pepsgo_peps P, const double* tensors, int on_device, void* stream) {
  if (!P || !tensors) return fail(PEPSGO_EINVAL, "pepsgo_peps_update: NULL argument");
  HIP_TRY(hipSetDevice(P->ctx->device));
  HIP_TRY(hipMemcpyAsync(P->dT, tensors, P->nparams * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         (hipStream_t)stream));
  return PEPSGO_OK;
}

int pepsgo_peps_read(pepsgo_peps P, double* tensors, int on_device, void* stream) {
  if (!P || !tensors) return fail(PEPSGO_EINVAL, "pepsgo_peps_read: NULL argument");
  HIP_TRY(hipSetDevice(P->ctx->device));
  HIP_TRY(hipMemcpyAsync(tensors, P->dT, P->nparams * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         (hipStream_t)stream));
  if (!on_device) HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return PEPSGO_OK;
}

int pepsgo_peps_free(pepsgo_peps P) {
  if (!P) return fail(PEPSGO_EINVAL, "pepsgo_peps_free: NULL handle");
  (void)hipSetDevice(P->ctx->device);
  (void)hipFree(P->dT);
  (void)hipFree(P->d_site_off);
  (void)hipFree(P->d_grad_off);
  (void)hipFree(P->d_ones);
  delete P;
  return PEPSGO_OK;
}

int pepsgo_grad_layout(pepsgo_peps P, int64_t* elems, int64_t* site_offsets) {
  if (!P || !elems) return fail(PEPSGO_EINVAL, "pepsgo_grad_layout: NULL argument");
  *elems = P->grad_elems;
  if (site_offsets) {
    for (size_t k = 0; k < P->grad_off.size(); ++k) site_offsets[k] = P->grad_off[k];
    site_offsets[P->grad_off.size()] = P->grad_elems;
  }
  return PEPSGO_OK;
}

static int check_params(const pepsgo_peps_* P, const pepsgo_eval_params* prm) {
  if (!prm) return fail(PEPSGO_EINVAL, "params is NULL");
  if (prm->Dc < 1) return fail(PEPSGO_EINVAL, "Dc = %d must be >= 1", prm->Dc);
  if (prm->Dc > PEPSGO_MAX_DC) return fail(PEPSGO_EUNSUPPORTED, "Dc = %d above %d", prm->Dc, PEPSGO_MAX_DC);
  if (prm->precision < PEPSGO_FP64 || prm->precision > PEPSGO_BF16)
    return fail(PEPSGO_EUNSUPPORTED, "precision %d is not supported", prm->precision);
  if (prm->grad_mode != PEPSGO_GRAD_NONE && prm->grad_mode != PEPSGO_GRAD_PER_SAMPLE &&
      prm->grad_mode != PEPSGO_GRAD_REDUCED)
    return fail(PEPSGO_EINVAL, "grad_mode %d unknown", prm->grad_mode);
  if (prm->grad_mode == PEPSGO_GRAD_REDUCED && !prm->want_eloc)
    return fail(PEPSGO_EINVAL, "grad_mode REDUCED needs want_eloc = 1 (the sums weigh Delta by E)");
  (void)P;
  return PEPSGO_OK;
}

int pepsgo_workspace_bytes(pepsgo_peps P, const pepsgo_eval_params* prm, int batch, size_t* bytes) {
  if (!P || !bytes) return fail(PEPSGO_EINVAL, "pepsgo_workspace_bytes: NULL argument");
  if (batch < 0) return fail(PEPSGO_EINVAL, "pepsgo_workspace_bytes: batch %d < 0", batch);
  int rc = check_params(P, prm);
  if (rc) return rc;
  const Plan p = make_plan(P, prm->Dc, prm->want_eloc, prm->precision,
                           tuning_for(P->ctx, P->D, prm->Dc, prm->precision), prm->grad_mode);
  *bytes = (size_t)p.ws_stride * sizeof(double) * (size_t)std::max(batch, 1);
  return PEPSGO_OK;
}

}  // extern "C"

// The launch sequence of one evaluation.  `timed`: bracket launches with
// profiling events when profiling is on (off inside a stream capture).
// Metropolis proposals riding on an evaluation (device arrays, per sample).
struct MetroArgs {
  const int32_t* bonds;
  const double* uniforms;
  uint8_t* configs;  // updated in place after the evaluation
  uint8_t* accepted;
};

// Bond dimensions of every boundary MPS and the zip shapes (the same for every
// sample of a batch), and the kernels' view of one evaluation.
struct Shapes {
  std::vector<std::vector<int>> top, bot;
  std::vector<ZipShape> ztop, zbot;
};

static Shapes make_shapes(const pepsgo_peps_* P, const Plan& p, const pepsgo_eval_params* prm) {
  (void)prm;
  const int N = p.N, M = p.M, D = p.D;
  Shapes sh;
  sh.bot.assign(N + 1, std::vector<int>(M + 1, 1));
  sh.top.assign(N, std::vector<int>(M + 1, 1));
  sh.zbot.resize(N);
  sh.ztop.resize(N);
  row_bonds(M, D, sh.bot[N - 1].data());
  for (int k = N - 2; k >= 1; --k) {
    sh.zbot[k] = make_zip(p, sh.bot[k + 1].data(), k, 1);
    for (int j = 0; j <= M; ++j) sh.bot[k][j] = sh.zbot[k].nb[j];
  }
  row_bonds(M, D, sh.top[0].data());
  for (int i = 1; i <= N - 2; ++i) {
    sh.ztop[i] = make_zip(p, sh.top[i - 1].data(), i, 0);
    for (int j = 0; j <= M; ++j) sh.top[i][j] = sh.ztop[i].nb[j];
  }
  (void)P;
  return sh;
}

static Lat make_lat(const pepsgo_peps_* P, const Plan& p, const pepsgo_eval_params* prm) {
  Lat L;
  L.N = p.N;
  L.M = p.M;
  L.D = p.D;
  L.Dc = prm->Dc;
  L.chimax = p.chimax;
  L.T = P->dT;
  L.site_off = P->d_site_off;
  L.cfg = nullptr;
  L.ws = nullptr;
  L.ws_stride = p.ws_stride;
  L.off_env = 0;
  L.env_stride = p.env_stride;
  L.site_slot = p.site_slot;
  L.off_envlog = p.off_envlog;
  L.off_rowlog = p.off_rowlog;
  L.off_rowsign = p.off_rowsign;
  L.off_eloc = p.off_eloc;
  L.off_flags = p.off_flags;
  L.off_re = p.off_re;
  L.re_slot = p.re_slot;
  L.off_re2 = p.off_re2;
  L.re2_slot = p.re2_slot;
  L.off_scratch = p.off_scratch;
  L.J1 = prm->J1;
  L.J2 = prm->J2;
  L.grad = nullptr;
  L.grad_stride = P->grad_elems;
  L.grad_off = P->d_grad_off;
  L.ones = P->d_ones;
  L.mbond = nullptr;
  return L;
}

static int evaluate_impl(pepsgo_peps P, const pepsgo_eval_params* prm, int batch,
                         const uint8_t* configs, double* logabs, int8_t* sign, double* eloc,
                         uint32_t* flags, double* grad, void* workspace, size_t workspace_bytes,
                         void* stream, bool timed, const MetroArgs* mh = nullptr) {
  if (!P) return fail(PEPSGO_EINVAL, "pepsgo_evaluate: NULL PEPS handle");
  int rc = check_params(P, prm);
  if (rc) return rc;
  if (batch < 0) return fail(PEPSGO_EINVAL, "pepsgo_evaluate: batch %d < 0", batch);
  if (batch == 0) return PEPSGO_OK;
  if (!configs || !logabs || !sign || !eloc || !flags || !workspace)
    return fail(PEPSGO_EINVAL, "pepsgo_evaluate: NULL buffer");
  if (prm->grad_mode != PEPSGO_GRAD_NONE && !grad)
    return fail(PEPSGO_EINVAL, "pepsgo_evaluate: grad_mode %s needs a grad buffer",
                prm->grad_mode == PEPSGO_GRAD_REDUCED ? "REDUCED" : "PER_SAMPLE");
  const Plan p = make_plan(P, prm->Dc, prm->want_eloc, prm->precision,
                           tuning_for(P->ctx, P->D, prm->Dc, prm->precision), prm->grad_mode);
  const size_t per = (size_t)p.ws_stride * sizeof(double);
  if (workspace_bytes < per)
    return fail(PEPSGO_EINVAL, "pepsgo_evaluate: workspace %zu bytes < %zu needed for one sample",
                workspace_bytes, per);
  const int chunk = (int)std::min<size_t>((size_t)batch, workspace_bytes / per);
  HIP_TRY(hipSetDevice(P->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int N = p.N, M = p.M, D = p.D;

  Shapes sh = make_shapes(P, p, prm);
  auto& top = sh.top;
  auto& bot = sh.bot;
  auto& ztop = sh.ztop;
  auto& zbot = sh.zbot;
  const int slot_tmp = N + 1;
  auto slotU = [&](int i) { return N - 1 + (i & 1); };  // U_i
  auto slotDn = [&](int k) { return k - 1; };             // Dn_k, k = 1..N-1
  Lat L = make_lat(P, p, prm);

  for (int b0 = 0; b0 < batch; b0 += chunk) {
    const int nb = std::min(chunk, batch - b0);
    L.cfg = configs + (int64_t)b0 * N * M;
    L.ws = reinterpret_cast<double*>(workspace);
    const bool reduced = prm->grad_mode == PEPSGO_GRAD_REDUCED;
    if (prm->grad_mode == PEPSGO_GRAD_PER_SAMPLE) {
      L.grad = grad + (int64_t)b0 * P->grad_elems;
      L.grad_stride = P->grad_elems;
    } else if (reduced) {
      // Delta blocks in the samples' workspace, summed below
      L.grad = reinterpret_cast<double*>(workspace) + p.off_grad;
      L.grad_stride = p.ws_stride;
    } else {
      L.grad = nullptr;
    }
    L.mbond = mh ? mh->bonds + b0 : nullptr;
    pepsgo_ctx_* C = P->ctx;
    {
      Timed t(C, PEPSGO_K_EDGES, s, timed);
      HIP_TRY(launch_edges(L, nb, slotU(0), slotDn(N - 1), 1, s));
    }
    for (int k = N - 2; k >= 1; --k) {
      ZipShape z = zbot[k];
      z.in_slot = slotDn(k + 1);
      z.out_slot = slotDn(k);
      z.tmp_slot = slot_tmp;
      Timed t(C, PEPSGO_K_ZIP, s, timed);
      HIP_TRY(launch_zip(L, z, p.zip, p.lds_zip, nb, s));
    }
    for (int i = 0; i < N; ++i) {
      SandShape sw;
      std::memset(&sw, 0, sizeof sw);
      sw.row = i;
      sw.top_slot = i == 0 ? -1 : slotU(i - 1);
      sw.bot_slot = i == N - 1 ? -1 : slotDn(i + 1);
      for (int j = 0; j <= M; ++j) {
        sw.ta[j] = i == 0 ? 1 : top[i - 1][j];
        sw.tb[j] = i == N - 1 ? 1 : bot[i + 1][j];
      }
      sw.want_grad = prm->grad_mode != PEPSGO_GRAD_NONE;
      sw.want_eloc = prm->want_eloc;
      {
        Timed t(C, PEPSGO_K_SANDWICH, s, timed);
        HIP_TRY(launch_sandwich(L, sw, p.sand, p.lds_sand, nb, s));
      }
      if (prm->want_eloc && i <= N - 2) {
        StripShape st;
        std::memset(&st, 0, sizeof st);
        st.row = i;
        st.top_slot = i == 0 ? -1 : slotU(i - 1);
        st.bot_slot = i + 2 <= N - 1 ? slotDn(i + 2) : -1;
        for (int j = 0; j <= M; ++j) {
          st.ta[j] = i == 0 ? 1 : top[i - 1][j];
          st.tb[j] = i + 2 <= N - 1 ? bot[i + 2][j] : 1;
        }
        st.want_diag = prm->J2 != 0.0;
        st.refine = 0;
        st.xc = p.xc;
        Timed t(C, PEPSGO_K_STRIP, s, timed);
        HIP_TRY(launch_strip(L, st, p.strip, p.lds_strip, nb, prm->precision, s));
        if (prm->precision != PEPSGO_FP64) {
          // float64 pass over the samples whose strip failed its accuracy check
          st.refine = 1;
          st.xc = p.xc64;
          HIP_TRY(launch_strip(L, st, p.strip64, p.lds_strip64, nb, PEPSGO_FP64, s));
        }
      }
      if (i >= 1 && i <= N - 2) {
        ZipShape z = ztop[i];
        z.in_slot = slotU(i - 1);
        z.out_slot = slotU(i);
        z.tmp_slot = slot_tmp;
        Timed t(C, PEPSGO_K_ZIP, s, timed);
        HIP_TRY(launch_zip(L, z, p.zip, p.lds_zip, nb, s));
      }
    }
    {
      Timed t(C, PEPSGO_K_FINALIZE, s, timed);
      HIP_TRY(launch_finalize(L, nb, prm->want_eloc, logabs + b0, sign + b0, eloc + b0, flags + b0, s));
    }
    if (reduced)  // Eq. (3) sums of this chunk, with the configurations before any move
      HIP_TRY(launch_go_accumulate(nb, N * M, P->grad_elems, p.ws_stride, L.cfg, L.grad, eloc + b0,
                                   flags + b0, P->d_grad_off, P->d_site_off, grad,
                                   grad + P->nparams, grad + 2 * P->nparams, s));
    if (mh)
      HIP_TRY(launch_metropolis(L, nb, mh->uniforms + b0, mh->configs + (int64_t)b0 * N * M,
                                mh->accepted + b0, s));
  }
  return PEPSGO_OK;
}

extern "C" {

int pepsgo_evaluate(pepsgo_peps P, const pepsgo_eval_params* prm, int batch, const uint8_t* configs,
                    double* logabs, int8_t* sign, double* eloc, uint32_t* flags, double* grad,
                    void* workspace, size_t workspace_bytes, void* stream) {
  return evaluate_impl(P, prm, batch, configs, logabs, sign, eloc, flags, grad, workspace,
                       workspace_bytes, stream, true);
}

int pepsgo_evaluate_noalloc(pepsgo_peps P, const pepsgo_eval_params* prm, int batch,
                            const uint8_t* configs, double* logabs, int8_t* sign, double* eloc,
                            uint32_t* flags, double* grad, void* stream) {
  if (!P) return fail(PEPSGO_EINVAL, "pepsgo_evaluate_noalloc: NULL PEPS handle");
  int rc = check_params(P, prm);
  if (rc) return rc;
  const Plan p = make_plan(P, prm->Dc, prm->want_eloc, prm->precision,
                           tuning_for(P->ctx, P->D, prm->Dc, prm->precision), prm->grad_mode);
  const size_t per = (size_t)p.ws_stride * sizeof(double);
  if (per > (size_t)PEPSGO_NOALLOC_SCRATCH_BYTES)
    return fail(PEPSGO_EUNSUPPORTED,
                "pepsgo_evaluate_noalloc: one sample of this shape needs %zu bytes of workspace, "
                "more than the fixed %zu-byte workspace; use pepsgo_evaluate with a caller workspace",
                per, (size_t)PEPSGO_NOALLOC_SCRATCH_BYTES);
  // no profiling events here (taking one may create it)
  return evaluate_impl(P, prm, batch, configs, logabs, sign, eloc, flags, grad, P->ctx->scratch,
                       (size_t)PEPSGO_NOALLOC_SCRATCH_BYTES, stream, false);
}

int pepsgo_metropolis_step(pepsgo_peps P, const pepsgo_eval_params* prm, int batch,
                           uint8_t* configs, const int32_t* bonds, const double* uniforms,
                           uint8_t* accepted, double* logabs, int8_t* sign, double* eloc,
                           uint32_t* flags, double* grad, void* workspace, size_t workspace_bytes,
                           void* stream) {
  if (!P || !prm) return fail(PEPSGO_EINVAL, "pepsgo_metropolis_step: NULL argument");
  if (!prm->want_eloc)
    return fail(PEPSGO_EINVAL, "pepsgo_metropolis_step: the exchange ratios come with want_eloc = 1");
  if (batch > 0 && (!bonds || !uniforms || !accepted))
    return fail(PEPSGO_EINVAL, "pepsgo_metropolis_step: NULL proposal buffer");
  MetroArgs mh{bonds, uniforms, configs, accepted};
  return evaluate_impl(P, prm, batch, configs, logabs, sign, eloc, flags, grad, workspace,
                       workspace_bytes, stream, true, &mh);
}

int pepsgo_metropolis_sweep(pepsgo_peps P, const pepsgo_eval_params* prm, int batch,
                            uint8_t* configs, const double* uniforms, uint8_t* accepted,
                            double* ratios, void* workspace, size_t workspace_bytes,
                            void* stream) {
  if (!P || !prm) return fail(PEPSGO_EINVAL, "pepsgo_metropolis_sweep: NULL argument");
  if (prm->Dc < 1) return fail(PEPSGO_EINVAL, "pepsgo_metropolis_sweep: Dc = %d must be >= 1", prm->Dc);
  if (prm->Dc > PEPSGO_MAX_DC)
    return fail(PEPSGO_EUNSUPPORTED, "pepsgo_metropolis_sweep: Dc = %d above %d", prm->Dc, PEPSGO_MAX_DC);
  if (batch < 0) return fail(PEPSGO_EINVAL, "pepsgo_metropolis_sweep: batch %d < 0", batch);
  if (batch == 0) return PEPSGO_OK;
  if (!configs || !uniforms || !accepted || !workspace)
    return fail(PEPSGO_EINVAL, "pepsgo_metropolis_sweep: NULL buffer");
  // decisions in float64 throughout: the plan of a float64 evaluation with energies
  pepsgo_eval_params q = *prm;
  q.precision = PEPSGO_FP64;
  q.grad_mode = PEPSGO_GRAD_NONE;
  q.want_eloc = 1;
  const Plan p = make_plan(P, q.Dc, 1, PEPSGO_FP64, tuning_for(P->ctx, P->D, q.Dc, PEPSGO_FP64));
  const size_t per = (size_t)p.ws_stride * sizeof(double);
  if (workspace_bytes < per)
    return fail(PEPSGO_EINVAL,
                "pepsgo_metropolis_sweep: workspace %zu bytes < %zu needed for one sample",
                workspace_bytes, per);
  const int chunk = (int)std::min<size_t>((size_t)batch, workspace_bytes / per);
  HIP_TRY(hipSetDevice(P->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int N = p.N, M = p.M;
  const int nbonds = N * (M - 1) + (N - 1) * M;
  Shapes sh = make_shapes(P, p, &q);
  const int slot_tmp = N + 1;
  auto slotU = [&](int i) { return N - 1 + (i & 1); };
  auto slotDn = [&](int k) { return k - 1; };
  Lat L = make_lat(P, p, &q);
  for (int b0 = 0; b0 < batch; b0 += chunk) {
    const int nb = std::min(chunk, batch - b0);
    uint8_t* cfg = configs + (int64_t)b0 * N * M;
    const double* un = uniforms + (int64_t)b0 * nbonds;
    uint8_t* acc = accepted + (int64_t)b0 * nbonds;
    double* rat = ratios ? ratios + (int64_t)b0 * nbonds : nullptr;
    L.cfg = cfg;
    L.ws = reinterpret_cast<double*>(workspace);
    HIP_TRY(launch_sweep_clear((int64_t)nb * nbonds, acc, rat, s));
    // bottom environments of the configurations as they are at the start
    HIP_TRY(launch_edges(L, nb, -1, slotDn(N - 1), 1, s));
    for (int k = N - 2; k >= 1; --k) {
      ZipShape z = sh.zbot[k];
      z.in_slot = slotDn(k + 1);
      z.out_slot = slotDn(k);
      z.tmp_slot = slot_tmp;
      HIP_TRY(launch_zip(L, z, p.zip, p.lds_zip, nb, s));
    }
    for (int i = 0; i < N; ++i) {
      const int k0 = i * (2 * M - 1);
      SandShape sw;
      std::memset(&sw, 0, sizeof sw);
      sw.row = i;
      sw.top_slot = i == 0 ? -1 : slotU(i - 1);
      sw.bot_slot = i == N - 1 ? -1 : slotDn(i + 1);
      for (int j = 0; j <= M; ++j) {
        sw.ta[j] = i == 0 ? 1 : sh.top[i - 1][j];
        sw.tb[j] = i == N - 1 ? 1 : sh.bot[i + 1][j];
      }
      HIP_TRY(launch_sweep_row(L, sw, p.sand, p.lds_sand, nb, cfg, un, acc, rat, nbonds, k0, s));
      if (i <= N - 2) {
        StripShape st;
        std::memset(&st, 0, sizeof st);
        st.row = i;
        st.top_slot = i == 0 ? -1 : slotU(i - 1);
        st.bot_slot = i + 2 <= N - 1 ? slotDn(i + 2) : -1;
        for (int j = 0; j <= M; ++j) {
          st.ta[j] = i == 0 ? 1 : sh.top[i - 1][j];
          st.tb[j] = i + 2 <= N - 1 ? sh.bot[i + 2][j] : 1;
        }
        st.xc = p.xc64;
        HIP_TRY(launch_sweep_strip(L, st, p.strip64, p.lds_strip64, nb, cfg, un, acc, rat, nbonds,
                                   k0, s));
      }
      // U_i of row i as it stands after its moves
      if (i == 0) HIP_TRY(launch_edges(L, nb, slotU(0), -1, 0, s));
      if (i >= 1 && i <= N - 2) {
        ZipShape z = sh.ztop[i];
        z.in_slot = slotU(i - 1);
        z.out_slot = slotU(i);
        z.tmp_slot = slot_tmp;
        HIP_TRY(launch_zip(L, z, p.zip, p.lds_zip, nb, s));
      }
    }
  }
  return PEPSGO_OK;
}

}  // extern "C"

// Workspace of the transverse pass.  Per sample: its own evaluation workspace
// (environments, psi_b per row), then h w instances, each with the slots of a
// top-environment chain (two ping-pong, one right-canonical temporary), a row
// sandwich's right environments, its ratios to later window sites and the
// kernels' global scratch, and h w instance configurations.
struct CorrPlan {
  Plan real, inst;
  int n;                 // window sites
  int64_t cfg_bytes;     // one instance configuration, padded
  size_t per_sample;     // bytes per sample of a chunk
};

static CorrPlan make_corr_plan(const pepsgo_peps_* P, const pepsgo_eval_params* prm, int h, int w) {
  CorrPlan c;
  c.real = make_plan(P, prm->Dc, 0, PEPSGO_FP64, tuning_for(P->ctx, P->D, prm->Dc, PEPSGO_FP64));
  const Plan& p = c.real;
  c.n = h * w;
  Plan q = p;
  q.n_env = 3;
  int64_t o = 3 * p.env_stride;
  q.off_envlog = o;
  o += 4;
  q.off_rowlog = o;
  o += round_up(p.N, 4);
  q.off_rowsign = o;
  o += round_up(p.N, 4);
  q.off_eloc = o;
  o += 4;
  q.off_flags = o;
  o += 4;
  q.off_re = o;
  o += (p.M + 1) * p.re_slot;
  q.off_re2 = o;
  q.re2_slot = 0;
  q.off_grad = o;  // the instance's ratio row
  o += round_up(c.n, 4);
  q.off_scratch = o;
  q.ws_stride = round_up(o + (p.ws_stride - p.off_scratch), 32);
  c.inst = q;
  c.cfg_bytes = round_up((int64_t)p.N * p.M, 8);
  c.per_sample = (size_t)p.ws_stride * 8 + (size_t)c.n * ((size_t)q.ws_stride * 8 + c.cfg_bytes);
  return c;
}

static int check_window(const char* fn, const pepsgo_peps_* P, int r0, int c0, int h, int w) {
  if (h < 1 || w < 1 || r0 < 0 || c0 < 0 || r0 + h > P->N || c0 + w > P->M)
    return fail(PEPSGO_EINVAL, "%s: window (%d,%d) %dx%d not inside %dx%d", fn, r0, c0, h, w, P->N,
                P->M);
  if (h * w > PEPSGO_MAX_WINDOW)
    return fail(PEPSGO_EUNSUPPORTED, "%s: window of %d sites above %d", fn, h * w,
                PEPSGO_MAX_WINDOW);
  return PEPSGO_OK;
}

extern "C" {

int pepsgo_transverse_workspace_bytes(pepsgo_peps P, const pepsgo_eval_params* prm, int r0, int c0,
                                      int h, int w, int batch, size_t* bytes) {
  if (!P || !prm || !bytes) return fail(PEPSGO_EINVAL, "pepsgo_transverse_workspace_bytes: NULL argument");
  int rc = check_params(P, prm);
  if (rc) return rc;
  rc = check_window("pepsgo_transverse_workspace_bytes", P, r0, c0, h, w);
  if (rc) return rc;
  if (batch < 0) return fail(PEPSGO_EINVAL, "pepsgo_transverse_workspace_bytes: batch %d < 0", batch);
  *bytes = make_corr_plan(P, prm, h, w).per_sample * (size_t)std::max(batch, 1);
  return PEPSGO_OK;
}

int pepsgo_transverse(pepsgo_peps P, const pepsgo_eval_params* prm, int batch,
                      const uint8_t* configs, int r0, int c0, int h, int w, double* ratios,
                      double* sums, int64_t* count, uint32_t* flags, void* workspace,
                      size_t workspace_bytes, void* stream) {
  if (!P || !prm) return fail(PEPSGO_EINVAL, "pepsgo_transverse: NULL argument");
  int rc = check_params(P, prm);
  if (rc) return rc;
  rc = check_window("pepsgo_transverse", P, r0, c0, h, w);
  if (rc) return rc;
  if (batch < 0) return fail(PEPSGO_EINVAL, "pepsgo_transverse: batch %d < 0", batch);
  if (batch == 0) return PEPSGO_OK;
  if (!configs || !sums || !count || !flags || !workspace)
    return fail(PEPSGO_EINVAL, "pepsgo_transverse: NULL buffer");
  pepsgo_eval_params q = *prm;
  q.precision = PEPSGO_FP64;
  q.grad_mode = PEPSGO_GRAD_NONE;
  q.want_eloc = 0;
  const CorrPlan cp = make_corr_plan(P, &q, h, w);
  if (workspace_bytes < cp.per_sample)
    return fail(PEPSGO_EINVAL, "pepsgo_transverse: workspace %zu bytes < %zu needed for one sample",
                workspace_bytes, cp.per_sample);
  const int chunk = (int)std::min<size_t>((size_t)batch, workspace_bytes / cp.per_sample);
  if ((int64_t)chunk * cp.n > (int64_t)INT32_MAX / 2)
    return fail(PEPSGO_EUNSUPPORTED, "pepsgo_transverse: %d instances in one chunk", chunk * cp.n);
  HIP_TRY(hipSetDevice(P->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const Plan& p = cp.real;
  const int N = p.N, M = p.M, n = cp.n;
  Shapes sh = make_shapes(P, p, &q);
  const int slot_tmp = N + 1;
  auto slotU = [&](int i) { return N - 1 + (i & 1); };
  auto slotDn = [&](int k) { return k - 1; };
  auto slotUv = [&](int i) { return i & 1; };  // instance chain; slot 2 is its temporary
  Lat R = make_lat(P, p, &q);
  Lat V = make_lat(P, cp.inst, &q);
  const int bmax = r0 + h - 1;
  for (int b0 = 0; b0 < batch; b0 += chunk) {
    const int nb = std::min(chunk, batch - b0);
    char* base = reinterpret_cast<char*>(workspace);
    R.cfg = configs + (int64_t)b0 * N * M;
    R.ws = reinterpret_cast<double*>(base);
    V.ws = reinterpret_cast<double*>(base + (size_t)nb * p.ws_stride * 8);
    uint8_t* icfg = reinterpret_cast<uint8_t*>(base + (size_t)nb * p.ws_stride * 8 +
                                               (size_t)nb * n * cp.inst.ws_stride * 8);
    V.cfg = icfg;
    FlipShape z;
    std::memset(&z, 0, sizeof z);
    z.r0 = r0;
    z.c0 = c0;
    z.h = h;
    z.w = w;
    z.nbr = nb;
    z.off_rat = cp.inst.off_grad;
    // the instance configurations are laid out [v][N*M] (unpadded): the
    // kernels index them with the lattice size
    HIP_TRY(launch_corr_init(V, z, n * nb, R.cfg, icfg, s));
    HIP_TRY(launch_edges(R, nb, slotU(0), slotDn(N - 1), 1, s));
    for (int k = N - 2; k >= std::max(1, r0 + 1); --k) {
      ZipShape zz = sh.zbot[k];
      zz.in_slot = slotDn(k + 1);
      zz.out_slot = slotDn(k);
      zz.tmp_slot = slot_tmp;
      HIP_TRY(launch_zip(R, zz, p.zip, p.lds_zip, nb, s));
    }
    for (int i = 0; i <= bmax; ++i) {
      if (i >= r0) {
        // psi_i(S) of the samples themselves
        SandShape sw;
        std::memset(&sw, 0, sizeof sw);
        sw.row = i;
        sw.top_slot = i == 0 ? -1 : slotU(i - 1);
        sw.bot_slot = i == N - 1 ? -1 : slotDn(i + 1);
        for (int j = 0; j <= M; ++j) {
          sw.ta[j] = i == 0 ? 1 : sh.top[i - 1][j];
          sw.tb[j] = i == N - 1 ? 1 : sh.bot[i + 1][j];
        }
        HIP_TRY(launch_sandwich(R, sw, p.sand, p.lds_sand, nb, s));
        const int xi = (i - r0) * w;  // first window index of row i
        const int active = (xi + w) * nb;
        if (i >= 1) HIP_TRY(launch_corr_copy(V, R, nb, xi * nb, w * nb, slotU(i - 1), slotUv(i - 1), s));
        z.row = i;
        z.top_slot = i == 0 ? -1 : slotUv(i - 1);
        z.bot_slot = i == N - 1 ? -1 : slotDn(i + 1);
        for (int j = 0; j <= M; ++j) {
          z.ta[j] = sw.ta[j];
          z.tb[j] = sw.tb[j];
        }
        HIP_TRY(launch_flip_row(V, R, z, p.sand, p.lds_sand, active, s));
        if (i < bmax) {
          if (i == 0) {
            HIP_TRY(launch_edges(V, active, slotUv(0), -1, 0, s));
          } else {
            ZipShape zz = sh.ztop[i];
            zz.in_slot = slotUv(i - 1);
            zz.out_slot = slotUv(i);
            zz.tmp_slot = 2;
            HIP_TRY(launch_zip(V, zz, p.zip, p.lds_zip, active, s));
          }
        }
      }
      if (i >= 1 && i < bmax && i <= N - 2) {
        ZipShape zz = sh.ztop[i];
        zz.in_slot = slotU(i - 1);
        zz.out_slot = slotU(i);
        zz.tmp_slot = slot_tmp;
        HIP_TRY(launch_zip(R, zz, p.zip, p.lds_zip, nb, s));
      }
    }
    HIP_TRY(launch_corr_finish(V, R, z, flags + b0, ratios ? ratios + (int64_t)b0 * n * n : nullptr,
                               sums, count, s));
  }
  return PEPSGO_OK;
}

int pepsgo_su_workspace_bytes(pepsgo_peps P, size_t* bytes) {
  if (!P || !bytes) return fail(PEPSGO_EINVAL, "pepsgo_su_workspace_bytes: NULL argument");
  *bytes = (size_t)su_workspace_doubles(P->N, P->M, P->D) * sizeof(double);
  return PEPSGO_OK;
}

int pepsgo_su_evolve(pepsgo_peps P, double* gamma, double* lambdas, double J1, double dtau,
                     int nsteps, void* workspace, size_t ws_bytes, void* stream) {
  if (!P || !gamma || !lambdas) return fail(PEPSGO_EINVAL, "pepsgo_su_evolve: NULL argument");
  if (nsteps < 0) return fail(PEPSGO_EINVAL, "pepsgo_su_evolve: nsteps %d < 0", nsteps);
  if (!std::isfinite(J1) || !std::isfinite(dtau))
    return fail(PEPSGO_EINVAL, "pepsgo_su_evolve: non-finite J1 or dtau");
  const size_t need = (size_t)su_workspace_doubles(P->N, P->M, P->D) * sizeof(double);
  if (nsteps == 0) return PEPSGO_OK;
  if (need > 0 && (!workspace || ws_bytes < need))
    return fail(PEPSGO_EINVAL, "pepsgo_su_evolve: workspace of %zu bytes, %zu needed", ws_bytes,
                need);
  // exp(-dtau J1 S.S): the singlet (S.S = -3/4) and the triplet (+1/4) projectors
  const double et = std::exp(-0.25 * dtau * J1), es = std::exp(0.75 * dtau * J1);
  double g[16] = {0};
  for (int k = 0; k < 4; ++k) g[5 * k] = et;
  const double ps[2][2] = {{0.5, -0.5}, {-0.5, 0.5}};  // singlet projector on {01, 10}
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) g[(1 + r) * 4 + 1 + c] += (es - et) * ps[r][c];
  HIP_TRY(hipSetDevice(P->ctx->device));
  for (int t = 0; t < nsteps; ++t)
    HIP_TRY(launch_su_step(P->N, P->M, P->D, gamma, P->d_site_off, lambdas,
                           static_cast<double*>(workspace), g, (hipStream_t)stream));
  return PEPSGO_OK;
}

int pepsgo_su_pad(pepsgo_peps from, const double* gamma, const double* lambdas, pepsgo_peps to,
                  double* gamma_out, double* lambdas_out, void* stream) {
  if (!from || !to || !gamma || !lambdas || !gamma_out || !lambdas_out)
    return fail(PEPSGO_EINVAL, "pepsgo_su_pad: NULL argument");
  if (from->N != to->N || from->M != to->M || to->D < from->D || from->ctx->device != to->ctx->device)
    return fail(PEPSGO_EINVAL,
                "pepsgo_su_pad: need the same lattice and device and D_to >= D_from "
                "(got %dx%d D=%d -> %dx%d D=%d)",
                from->N, from->M, from->D, to->N, to->M, to->D);
  HIP_TRY(hipSetDevice(to->ctx->device));
  HIP_TRY(launch_su_pad(to->N, to->M, from->D, to->D, from->d_site_off, to->d_site_off,
                        to->nparams, gamma, gamma_out, lambdas, lambdas_out, (hipStream_t)stream));
  return PEPSGO_OK;
}

int pepsgo_su_to_peps(pepsgo_peps P, const double* gamma, const double* lambdas, void* stream) {
  if (!P || !gamma || !lambdas) return fail(PEPSGO_EINVAL, "pepsgo_su_to_peps: NULL argument");
  HIP_TRY(hipSetDevice(P->ctx->device));
  HIP_TRY(launch_su_absorb(P->N, P->M, P->D, gamma, P->d_site_off, lambdas, P->nparams, P->dT,
                           (hipStream_t)stream));
  return PEPSGO_OK;
}

int pepsgo_sz_counts(int nrows, int ncols, int r0, int c0, int h, int w, int batch,
                     const uint8_t* configs, const uint32_t* flags, int64_t* same,
                     int64_t* nsamples, void* stream) {
  if (nrows < 1 || ncols < 1 || nrows > kMaxSide || ncols > kMaxSide)
    return fail(PEPSGO_EINVAL, "pepsgo_sz_counts: lattice %dx%d outside 1..%d", nrows, ncols,
                kMaxSide);
  if (h < 1 || w < 1 || r0 < 0 || c0 < 0 || r0 + h > nrows || c0 + w > ncols)
    return fail(PEPSGO_EINVAL, "pepsgo_sz_counts: window (%d,%d) %dx%d not inside %dx%d", r0, c0,
                h, w, nrows, ncols);
  if (batch < 0) return fail(PEPSGO_EINVAL, "pepsgo_sz_counts: batch %d < 0", batch);
  if (!same || !nsamples || (batch > 0 && !configs))
    return fail(PEPSGO_EINVAL, "pepsgo_sz_counts: NULL buffer");
  if (batch == 0) return PEPSGO_OK;
  HIP_TRY(launch_sz_counts(nrows, ncols, r0, c0, h, w, batch, configs, flags, same, nsamples,
                           (hipStream_t)stream));
  return PEPSGO_OK;
}

int pepsgo_structure_factor(int h, int w, const int64_t* same, const int64_t* nsamples, double kx,
                            double ky, double factor, double* out, void* stream) {
  if (h < 1 || w < 1 || h > kMaxSide || w > kMaxSide)
    return fail(PEPSGO_EINVAL, "pepsgo_structure_factor: window %dx%d outside 1..%d", h, w,
                kMaxSide);
  if (!same || !nsamples || !out) return fail(PEPSGO_EINVAL, "pepsgo_structure_factor: NULL buffer");
  HIP_TRY(launch_structure_factor(h, w, same, nsamples, nullptr, nullptr, kx, ky, factor, out,
                                  (hipStream_t)stream));
  return PEPSGO_OK;
}

int pepsgo_spin_structure_factor(int h, int w, const int64_t* same, const int64_t* nsamples,
                                 const double* trans, const int64_t* ntrans, double kx, double ky,
                                 double* out, void* stream) {
  if (h < 1 || w < 1 || h > kMaxSide || w > kMaxSide)
    return fail(PEPSGO_EINVAL, "pepsgo_spin_structure_factor: window %dx%d outside 1..%d", h, w,
                kMaxSide);
  if (!same || !nsamples || !trans || !ntrans || !out)
    return fail(PEPSGO_EINVAL, "pepsgo_spin_structure_factor: NULL buffer");
  HIP_TRY(launch_structure_factor(h, w, same, nsamples, trans, ntrans, kx, ky, 1.0, out,
                                  (hipStream_t)stream));
  return PEPSGO_OK;
}

int pepsgo_go_accumulate(pepsgo_peps P, int batch, const uint8_t* configs, const double* grad,
                         const double* eloc, const uint32_t* flags, double* sum_delta,
                         double* sum_delta_e, double* stats, void* stream) {
  if (!P) return fail(PEPSGO_EINVAL, "pepsgo_go_accumulate: NULL PEPS handle");
  if (batch < 0) return fail(PEPSGO_EINVAL, "pepsgo_go_accumulate: batch %d < 0", batch);
  if (batch == 0) return PEPSGO_OK;
  if (!configs || !grad || !eloc || !flags || !sum_delta || !sum_delta_e || !stats)
    return fail(PEPSGO_EINVAL, "pepsgo_go_accumulate: NULL buffer");
  HIP_TRY(hipSetDevice(P->ctx->device));
  HIP_TRY(launch_go_accumulate(batch, P->N * P->M, P->grad_elems, P->grad_elems, configs, grad,
                               eloc, flags, P->d_grad_off, P->d_site_off, sum_delta, sum_delta_e,
                               stats, (hipStream_t)stream));
  return PEPSGO_OK;
}

int pepsgo_go_update(pepsgo_peps P, const double* sum_delta, const double* sum_delta_e,
                     const double* stats, double dt, const double* p, void* stream) {
  if (!P || !sum_delta || !sum_delta_e || !stats || !p)
    return fail(PEPSGO_EINVAL, "pepsgo_go_update: NULL argument");
  if (!(dt >= 0.0)) return fail(PEPSGO_EINVAL, "pepsgo_go_update: step %g must be >= 0", dt);
  HIP_TRY(hipSetDevice(P->ctx->device));
  HIP_TRY(launch_go_update(P->nparams, P->dT, sum_delta, sum_delta_e, stats, dt, p,
                           (hipStream_t)stream));
  return PEPSGO_OK;
}

int pepsgo_graph_create(pepsgo_peps P, const pepsgo_eval_params* prm, int batch,
                        const uint8_t* configs, double* logabs, int8_t* sign, double* eloc,
                        uint32_t* flags, double* grad, void* workspace, size_t workspace_bytes,
                        pepsgo_graph* out) {
  if (!P || !prm || !out) return fail(PEPSGO_EINVAL, "pepsgo_graph_create: NULL argument");
  int rc = check_params(P, prm);
  if (rc) return rc;
  if (batch < 1) return fail(PEPSGO_EINVAL, "pepsgo_graph_create: batch %d < 1", batch);
  HIP_TRY(hipSetDevice(P->ctx->device));
  const Plan p = make_plan(P, prm->Dc, prm->want_eloc, prm->precision,
                           tuning_for(P->ctx, P->D, prm->Dc, prm->precision), prm->grad_mode);
  // kernel attributes are set outside the capture
  HIP_TRY(prepare_lds(p.lds_zip, p.lds_sand, p.lds_strip, prm->precision));
  HIP_TRY(prepare_lds(p.lds_zip, p.lds_sand, p.lds_strip64, PEPSGO_FP64));
  hipStream_t s;
  HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(s);
    return fail(PEPSGO_EDEVICE, "pepsgo_graph_create: hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  rc = evaluate_impl(P, prm, batch, configs, logabs, sign, eloc, flags, grad, workspace,
                     workspace_bytes, s, false);
  e = hipStreamEndCapture(s, &g);
  (void)hipStreamDestroy(s);
  if (rc != PEPSGO_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(PEPSGO_EDEVICE, "pepsgo_graph_create: capture: %s", hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(PEPSGO_EDEVICE, "pepsgo_graph_create: instantiate: %s", hipGetErrorString(e));
  }
  auto* G = new pepsgo_graph_;
  G->device = P->ctx->device;
  G->graph = g;
  G->exec = x;
  *out = G;
  return PEPSGO_OK;
}

int pepsgo_graph_launch(pepsgo_graph G, void* stream) {
  if (!G) return fail(PEPSGO_EINVAL, "pepsgo_graph_launch: NULL graph");
  HIP_TRY(hipSetDevice(G->device));
  HIP_TRY(hipGraphLaunch(G->exec, (hipStream_t)stream));
  return PEPSGO_OK;
}

int pepsgo_graph_free(pepsgo_graph G) {
  if (!G) return fail(PEPSGO_EINVAL, "pepsgo_graph_free: NULL graph");
  (void)hipSetDevice(G->device);
  (void)hipGraphExecDestroy(G->exec);
  (void)hipGraphDestroy(G->graph);
  delete G;
  return PEPSGO_OK;
}


int pepsgo_tune_get(pepsgo_ctx ctx, int D, int Dc, int precision, pepsgo_tuning* out) {
  if (!ctx || !out) return fail(PEPSGO_EINVAL, "pepsgo_tune_get: NULL argument");
  *out = tuning_for(ctx, D, Dc, precision);
  return PEPSGO_OK;
}

int pepsgo_tune_set(pepsgo_ctx ctx, int D, int Dc, int precision, const pepsgo_tuning* t) {
  if (!ctx) return fail(PEPSGO_EINVAL, "pepsgo_tune_set: NULL context");
  if (t && (t->zip_lds_bytes < 0 || t->sandwich_lds_bytes < 0 || t->strip_lds_bytes < 0 ||
            t->strip_xc < 0))
    return fail(PEPSGO_EINVAL, "pepsgo_tune_set: negative budget");
  std::lock_guard<std::mutex> g(ctx->tune_mu);
  const auto key = std::make_tuple(D, Dc, precision);
  if (!t) {
    ctx->tune.erase(key);
    return PEPSGO_OK;
  }
  pepsgo_tuning v = default_tuning(precision, ctx->lds_budget);
  if (t->zip_lds_bytes) v.zip_lds_bytes = std::min(t->zip_lds_bytes, ctx->lds_budget);
  if (t->sandwich_lds_bytes) v.sandwich_lds_bytes = std::min(t->sandwich_lds_bytes, ctx->lds_budget);
  if (t->strip_lds_bytes) v.strip_lds_bytes = std::min(t->strip_lds_bytes, ctx->lds_budget);
  if (t->strip_xc) v.strip_xc = std::max(1, std::min(4, t->strip_xc));
  ctx->tune[key] = v;
  return PEPSGO_OK;
}

int pepsgo_autotune(pepsgo_peps P, const pepsgo_eval_params* prm, int batch, const uint8_t* configs,
                    void* stream, pepsgo_tuning* chosen) {
  if (!P || !configs) return fail(PEPSGO_EINVAL, "pepsgo_autotune: NULL argument");
  int rc = check_params(P, prm);
  if (rc) return rc;
  if (batch < 1) return fail(PEPSGO_EINVAL, "pepsgo_autotune: batch %d < 1", batch);
  pepsgo_ctx_* C = P->ctx;
  const int lb = C->lds_budget;
  // candidate budgets: five, four, three, two and one workgroups per CU (five
  // of four waves fit the registers of the strip and the sandwich); for the
  // strip also 2 or 3 x values per stage
  const std::vector<std::pair<int, int>> cand = {
      {std::min(lb, 32 * 1024), 1}, {std::min(lb, 40 * 1024), 1}, {std::min(lb, 53 * 1024), 1},
      {std::min(lb, 80 * 1024), 1},
      {lb, 1},                      {std::min(lb, 80 * 1024), 2}, {lb, 2},
      {lb, 3}};
  // truncation: one-wave workgroups at 20 or 40 KB (blocks up to 72 x 72), four-wave ones at 80 KB
  // or the whole budget
  std::vector<int> zc = {std::min(lb, 80 * 1024), lb};
  if ((int64_t)std::max(prm->Dc, P->D) * P->D <= 72) zc = {20 * 1024, 40 * 1024, std::min(lb, 80 * 1024), lb};
  const std::vector<int> sc = {std::min(lb, 32 * 1024), std::min(lb, 40 * 1024),
                               std::min(lb, 53 * 1024), std::min(lb, 80 * 1024), lb};
  const int rows = (int)std::max({cand.size(), zc.size(), sc.size()});
  auto pick = [](const auto& v, int r) { return v[std::min<size_t>(r, v.size() - 1)]; };
  auto row_tuning = [&](int r) {
    return pepsgo_tuning{pick(zc, r), pick(sc, r), pick(cand, r).first, pick(cand, r).second};
  };
  size_t ws_max = 0;
  for (int r = 0; r < rows; ++r) {
    pepsgo_tuning t = row_tuning(r);
    const Plan p = make_plan(P, prm->Dc, prm->want_eloc, prm->precision, t, prm->grad_mode);
    ws_max = std::max(ws_max, (size_t)p.ws_stride * 8 * (size_t)batch);
  }
  HIP_TRY(hipSetDevice(C->device));
  const bool g = prm->grad_mode == PEPSGO_GRAD_PER_SAMPLE;
  const bool gr_sums = prm->grad_mode == PEPSGO_GRAD_REDUCED;
  char* mem = nullptr;
  const size_t gbytes = g ? (size_t)batch * P->grad_elems * 8
                          : (gr_sums ? (size_t)(2 * P->nparams + 3) * 8 : 0);
  const size_t out_bytes = (size_t)batch * (8 + 8 + 4 + 1 + 7) + gbytes;
  if (hipMalloc(&mem, ws_max + out_bytes + 1024) != hipSuccess) {
    (void)hipGetLastError();
    return fail(PEPSGO_ENOMEM, "pepsgo_autotune: cannot allocate %zu bytes", ws_max + out_bytes);
  }
  char* o = mem + round_up((int64_t)ws_max, 256);
  double* la = reinterpret_cast<double*>(o);
  double* el = la + batch;
  double* gr = (g || gr_sums) ? el + batch : nullptr;
  uint32_t* fl = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(el + batch) + gbytes);
  int8_t* sg = reinterpret_cast<int8_t*>(fl + batch);
  const auto key = std::make_tuple(P->D, prm->Dc, prm->precision);
  pepsgo_tuning prev;
  bool had;
  {
    std::lock_guard<std::mutex> gl(C->tune_mu);
    auto it = C->tune.find(key);
    had = it != C->tune.end();
    if (had) prev = it->second;
  }
  const int prof_prev = C->profiling;
  double best[3] = {1e300, 1e300, 1e300};
  pepsgo_tuning win = default_tuning(prm->precision, lb);
  const int cls[3] = {PEPSGO_K_ZIP, PEPSGO_K_SANDWICH, PEPSGO_K_STRIP};
  rc = PEPSGO_OK;
  for (int r = -1; r < rows && rc == PEPSGO_OK; ++r) {  // r = -1: untimed warm-up
    pepsgo_tuning t = r < 0 ? default_tuning(prm->precision, lb) : row_tuning(r);
    {
      std::lock_guard<std::mutex> gl(C->tune_mu);
      C->tune[key] = t;
    }
    pepsgo_profile(C, -1);
    C->profiling = r >= 0;
    rc = pepsgo_evaluate(P, prm, batch, configs, la, sg, el, fl, gr, mem, ws_max, stream);
    C->profiling = prof_prev;
    if (rc != PEPSGO_OK) break;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
      rc = fail(PEPSGO_EDEVICE, "pepsgo_autotune: evaluation failed on the device");
      break;
    }
    if (r < 0) continue;
    for (int k = 0; k < 3; ++k) {
      double ms;
      int64_t n;
      pepsgo_profile_read(C, cls[k], &ms, &n);
      if (n > 0 && ms < best[k]) {
        best[k] = ms;
        if (k == 0) win.zip_lds_bytes = t.zip_lds_bytes;
        if (k == 1) win.sandwich_lds_bytes = t.sandwich_lds_bytes;
        if (k == 2) {
          win.strip_lds_bytes = t.strip_lds_bytes;
          win.strip_xc = t.strip_xc;
        }
      }
    }
  }
  pepsgo_profile(C, -1);
  (void)hipFree(mem);
  {
    std::lock_guard<std::mutex> gl(C->tune_mu);
    if (rc == PEPSGO_OK)
      C->tune[key] = win;
    else if (had)
      C->tune[key] = prev;
    else
      C->tune.erase(key);
  }
  if (rc == PEPSGO_OK && chosen) *chosen = win;
  return rc;
}

static std::string arch_name(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

int pepsgo_tune_save(pepsgo_ctx ctx, const char* path) {
  if (!ctx || !path) return fail(PEPSGO_EINVAL, "pepsgo_tune_save: NULL argument");
  FILE* f = fopen(path, "w");
  if (!f) return fail(PEPSGO_EINVAL, "pepsgo_tune_save: cannot write %s", path);
  fprintf(f, "# pepsgo tuning v2 %s\n", arch_name(ctx->device).c_str());
  std::lock_guard<std::mutex> g(ctx->tune_mu);
  for (const auto& kv : ctx->tune)
    fprintf(f, "%d %d %d %d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first),
            std::get<2>(kv.first), kv.second.zip_lds_bytes, kv.second.sandwich_lds_bytes,
            kv.second.strip_lds_bytes, kv.second.strip_xc);
  fclose(f);
  return PEPSGO_OK;
}

int pepsgo_tune_load(pepsgo_ctx ctx, const char* path) {
  if (!ctx || !path) return fail(PEPSGO_EINVAL, "pepsgo_tune_load: NULL argument");
  FILE* f = fopen(path, "r");
  if (!f) return fail(PEPSGO_EINVAL, "pepsgo_tune_load: cannot read %s", path);
  char line[256];
  int n = 0;
  bool ok = false;
  const std::string want = "# pepsgo tuning v2 " + arch_name(ctx->device);
  if (fgets(line, sizeof line, f)) {
    std::string h(line);
    while (!h.empty() && (h.back() == '\n' || h.back() == '\r')) h.pop_back();
    ok = h == want;
  }
  while (ok && fgets(line, sizeof line, f)) {
    int D, Dc, pr;
    pepsgo_tuning t;
    if (sscanf(line, "%d %d %d %d %d %d %d", &D, &Dc, &pr, &t.zip_lds_bytes, &t.sandwich_lds_bytes,
               &t.strip_lds_bytes, &t.strip_xc) == 7 &&
        pepsgo_tune_set(ctx, D, Dc, pr, &t) == PEPSGO_OK)
      ++n;
  }
  fclose(f);
  return n;
}

}  // extern "C"
