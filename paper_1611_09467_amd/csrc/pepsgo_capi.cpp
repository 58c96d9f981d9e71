// Host side of the C-ABI: argument checks, shape planning, workspace layout and
// the launch sequence of one evaluation (see include/pepsgo.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
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

struct pepsgo_ctx_ {
  int device;
  int lds_budget;  // bytes of LDS a workgroup may use
  int profiling = 0;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;         // events recorded since the last read/reset
  std::vector<hipEvent_t> pool;  // reusable events
  double total_ms[PEPSGO_K_COUNT] = {0};
  int64_t launches[PEPSGO_K_COUNT] = {0};
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
  int64_t off_envlog, off_rowlog, off_rowsign, off_eloc, off_flags, off_re, off_re2, off_scratch;
  int64_t ws_stride;  // doubles
  BufPlan zip, sand, strip;
  int lds_zip, lds_sand, lds_strip;
  int eig_batch;
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

Plan make_plan(const pepsgo_peps_* P, int Dc, int want_eloc) {
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
  p.off_scratch = o;

  const int budget = P->ctx->lds_budget;
  const int64_t red = kThreads + 2 * (kMaxSide + 1);
  const int64_t rowsmax = chi * D;
  // truncation kernel: Gram matrix, eigensolver work and carry in LDS; X in the
  // sample's global scratch; two workgroups per CU when they fit in 80 KB
  std::vector<int64_t> zs(ZB_COUNT);
  zs[ZB_RED] = 64;
  zs[ZB_MISC] = 4 * chi + 8;
  zs[ZB_G] = std::max({rowsmax * rowsmax, chi * D * D * chi, chi * D * chi});
  // eigensolver work followed by the eigenvectors; also the LQ reflectors and a staged MPS tensor
  zs[ZB_V] = std::max<int64_t>(sym_top_eig_work((int)rowsmax, (int)chi, kZipThreads) + rowsmax * chi,
                               chi * D * chi);
  zs[ZB_C] = std::max(chi * chi * D, 2 * chi * chi);
  zs[ZB_X] = std::max(rowsmax * rowsmax, chi * D * chi);
  const int64_t lw_min =
      std::max({chi * D * chi, D * D * D * D, 3 * rowsmax + chi, (int64_t)2 * kZipThreads});
  auto round4 = [](int64_t v) { return round_up(v, 4); };
  const int64_t fixed = round4(zs[ZB_RED]) + round4(zs[ZB_MISC]) + round4(zs[ZB_G]) +
                        round4(zs[ZB_V]) + round4(zs[ZB_C]);
  int zbudget = std::min(budget, 80 * 1024);
  if ((fixed + round4(lw_min)) * 8 > zbudget) zbudget = budget;
  int64_t lw = std::max(lw_min, std::min<int64_t>(3 * rowsmax * chi + chi, zbudget / 8 - fixed - 4));
  p.eig_batch = (int)std::max<int64_t>(1, std::min<int64_t>(chi, (lw - chi) / (3 * rowsmax)));
  zs[ZB_LW] = lw;
  std::vector<int> zorder = {ZB_RED, ZB_MISC, ZB_G, ZB_V, ZB_C, ZB_LW, ZB_X};
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
    gs = place(sz, budget, &tmp, &p.lds_sand);
    p.sand.glob = 0;
    for (size_t q = 0; q < sorder.size(); ++q) {
      p.sand.off[sorder[q]] = tmp.off[q];
      if ((tmp.glob >> q) & 1u) p.sand.glob |= 1u << sorder[q];
    }
  }
  std::vector<int64_t> ts(TB_COUNT);
  ts[TB_RED] = red;
  // odd leading dimensions of the strip intermediates
  const int64_t ld1 = (D * D) | 1, ld3 = (chi * D) | 1;
  ts[TB_T1] = std::max(D * chi * ld1, D * D * ld3);  // also holds the third intermediate
  ts[TB_T2] = chi * D * ld1;
  ts[TB_STG] = 2 * chi * D * chi + 2 * D * D * D * D;
  ts[TB_LE0] = chi * D * D * chi;
  ts[TB_LE1] = chi * D * D * chi;
  ts[TB_E1] = chi * D * D * chi;
  ts[TB_E2] = chi * D * D * chi;
  // the strip keeps only its per-x intermediates in LDS so two workgroups share a CU
  int64_t gt = want_eloc ? place(ts, std::min(budget, 80 * 1024), &p.strip, &p.lds_strip) : 0;
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
  return z;
}

// Bracket one launch with events when profiling is on.
struct Timed {
  pepsgo_ctx_* c;
  int cls;
  hipStream_t s;
  hipEvent_t a{}, b{};
  Timed(pepsgo_ctx_* c_, int cls_, hipStream_t s_) : c(c_), cls(cls_), s(s_) {
    if (!c->profiling) return;
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
    if (!c->profiling) return;
    (void)hipEventRecord(b, s);
    c->recs.push_back({cls, a, b});
  }
};

void drain_profile(pepsgo_ctx_* c) {
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

int pepsgo_create(int hip_device, pepsgo_ctx* out) {
  if (!out) return fail(PEPSGO_EINVAL, "pepsgo_create: out is NULL");
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n)
    return fail(PEPSGO_EINVAL, "pepsgo_create: device %d out of range (%d devices)", hip_device, n);
  HIP_TRY(hipSetDevice(hip_device));
  int lds = 0;
  HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device));
  auto* c = new pepsgo_ctx_;
  c->device = hip_device;
  c->lds_budget = std::min(lds, 160 * 1024);
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
    return fail(PEPSGO_EUNSUPPORTED, "precision %d not available in this build", prm->precision);
  if (prm->grad_mode != PEPSGO_GRAD_NONE && prm->grad_mode != PEPSGO_GRAD_PER_SAMPLE)
    return fail(PEPSGO_EINVAL, "grad_mode %d unknown", prm->grad_mode);
  (void)P;
  return PEPSGO_OK;
}

int pepsgo_workspace_bytes(pepsgo_peps P, const pepsgo_eval_params* prm, int batch, size_t* bytes) {
  if (!P || !bytes) return fail(PEPSGO_EINVAL, "pepsgo_workspace_bytes: NULL argument");
  if (batch < 0) return fail(PEPSGO_EINVAL, "pepsgo_workspace_bytes: batch %d < 0", batch);
  int rc = check_params(P, prm);
  if (rc) return rc;
  const Plan p = make_plan(P, prm->Dc, prm->want_eloc);
  *bytes = (size_t)p.ws_stride * sizeof(double) * (size_t)std::max(batch, 1);
  return PEPSGO_OK;
}

int pepsgo_evaluate(pepsgo_peps P, const pepsgo_eval_params* prm, int batch, const uint8_t* configs,
                    double* logabs, int8_t* sign, double* eloc, uint32_t* flags, double* grad,
                    void* workspace, size_t workspace_bytes, void* stream) {
  if (!P) return fail(PEPSGO_EINVAL, "pepsgo_evaluate: NULL PEPS handle");
  int rc = check_params(P, prm);
  if (rc) return rc;
  if (batch < 0) return fail(PEPSGO_EINVAL, "pepsgo_evaluate: batch %d < 0", batch);
  if (batch == 0) return PEPSGO_OK;
  if (!configs || !logabs || !sign || !eloc || !flags || !workspace)
    return fail(PEPSGO_EINVAL, "pepsgo_evaluate: NULL buffer");
  if (prm->grad_mode == PEPSGO_GRAD_PER_SAMPLE && !grad)
    return fail(PEPSGO_EINVAL, "pepsgo_evaluate: grad_mode PER_SAMPLE needs a grad buffer");
  const Plan p = make_plan(P, prm->Dc, prm->want_eloc);
  const size_t per = (size_t)p.ws_stride * sizeof(double);
  if (workspace_bytes < per)
    return fail(PEPSGO_EINVAL, "pepsgo_evaluate: workspace %zu bytes < %zu needed for one sample",
                workspace_bytes, per);
  const int chunk = (int)std::min<size_t>((size_t)batch, workspace_bytes / per);
  HIP_TRY(hipSetDevice(P->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int N = p.N, M = p.M, D = p.D;

  // boundary-MPS bond dimensions (identical for every sample)
  std::vector<std::vector<int>> bot(N + 1, std::vector<int>(M + 1, 1)), top(N, std::vector<int>(M + 1, 1));
  std::vector<ZipShape> zbot(N), ztop(N);
  row_bonds(M, D, bot[N - 1].data());
  for (int k = N - 2; k >= 1; --k) {
    zbot[k] = make_zip(p, bot[k + 1].data(), k, 1);
    for (int j = 0; j <= M; ++j) bot[k][j] = zbot[k].nb[j];
  }
  row_bonds(M, D, top[0].data());
  for (int i = 1; i <= N - 2; ++i) {
    ztop[i] = make_zip(p, top[i - 1].data(), i, 0);
    for (int j = 0; j <= M; ++j) top[i][j] = ztop[i].nb[j];
  }
  const int slot_tmp = N + 1;
  auto slotU = [&](int i) { return N - 1 + (i & 1); };  // U_i
  auto slotDn = [&](int k) { return k - 1; };             // Dn_k, k = 1..N-1

  Lat L;
  L.N = N;
  L.M = M;
  L.D = D;
  L.Dc = prm->Dc;
  L.chimax = p.chimax;
  L.T = P->dT;
  L.site_off = P->d_site_off;
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
  L.grad_stride = P->grad_elems;
  L.grad_off = P->d_grad_off;
  L.ones = P->d_ones;

  for (int b0 = 0; b0 < batch; b0 += chunk) {
    const int nb = std::min(chunk, batch - b0);
    L.cfg = configs + (int64_t)b0 * N * M;
    L.ws = reinterpret_cast<double*>(workspace);
    L.grad = prm->grad_mode == PEPSGO_GRAD_PER_SAMPLE ? grad + (int64_t)b0 * P->grad_elems : nullptr;
    pepsgo_ctx_* C = P->ctx;
    {
      Timed t(C, PEPSGO_K_EDGES, s);
      HIP_TRY(launch_edges(L, nb, slotU(0), slotDn(N - 1), s));
    }
    for (int k = N - 2; k >= 1; --k) {
      ZipShape z = zbot[k];
      z.in_slot = slotDn(k + 1);
      z.out_slot = slotDn(k);
      z.tmp_slot = slot_tmp;
      Timed t(C, PEPSGO_K_ZIP, s);
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
      sw.want_grad = prm->grad_mode == PEPSGO_GRAD_PER_SAMPLE;
      sw.want_eloc = prm->want_eloc;
      {
        Timed t(C, PEPSGO_K_SANDWICH, s);
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
        Timed t(C, PEPSGO_K_STRIP, s);
        HIP_TRY(launch_strip(L, st, p.strip, p.lds_strip, nb, prm->precision, s));
      }
      if (i >= 1 && i <= N - 2) {
        ZipShape z = ztop[i];
        z.in_slot = slotU(i - 1);
        z.out_slot = slotU(i);
        z.tmp_slot = slot_tmp;
        Timed t(C, PEPSGO_K_ZIP, s);
        HIP_TRY(launch_zip(L, z, p.zip, p.lds_zip, nb, s));
      }
    }
    Timed t(C, PEPSGO_K_FINALIZE, s);
    HIP_TRY(launch_finalize(L, nb, prm->want_eloc, logabs + b0, sign + b0, eloc + b0, flags + b0, s));
  }
  return PEPSGO_OK;
}

}  // extern "C"
