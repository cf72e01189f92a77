// hfqmc_abi.cpp -- host side of the C ABI declared in include/hfqmc.h.
//
// Validates problems, computes the HS coupling, plans the batch (one kernel
// class per padded slice count), lays out the caller's workspace, launches
// the gfx950 kernels on the context stream and finalises bin statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hfqmc.h"
#include "hfqmc_internal.h"

namespace hfqmc {
struct KernelInfo;
const KernelInfo* find_kernel(int LT, int RT, int DK);
int kernel_threads(const KernelInfo* k);
size_t kernel_lds(const KernelInfo* k);
hipError_t kernel_occupancy(const KernelInfo* k, int* blocks_per_cu);
hipError_t launch_sweep(const KernelInfo* k, int grid, hipStream_t st, const ImpDesc* descs, const int32_t* order,
                        int n_items, int* queue, uint8_t* ws);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
}  // namespace hfqmc

using namespace hfqmc;

namespace {

thread_local std::string t_err;

hfqmc_status fail(hfqmc_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
hfqmc_status fail(hfqmc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return fail(HFQMC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int padded_L(int L) { return (L + 15) / 16 * 16; }

// Tile-rows per wave for a padded slice count and update kind (environment
// override for tuning experiments).
int choose_rt(int LT, int DK = 0) {
  const char* e = getenv("HFQMC_RT");
  if (e && DK == 0) {
    int rt = strcmp(e, "max") == 0 ? LT / 16 : atoi(e);
    if (find_kernel(LT, rt, 0)) return rt;
  }
  return LT == 64 ? 2 : 1;
}

// Update kind of a problem: 0 plain rank-one, 1 delayed fp64, 2 delayed mixed.
int update_kind(const hfqmc_problem& p, hfqmc_precision prec) {
  const int k = p.delay == 0 ? 1 : p.delay;
  if (k <= 1) return 0;
  return prec == HFQMC_MIXED ? 2 : 1;
}

// HS coupling from cosh(lambda) = exp(dtau U / 2), written as
// acosh(1 + m) = log1p(m + sqrt(m (m + 2))) with m = expm1(dtau U / 2).
double coupling(double dtau, double U) {
  const double m = std::expm1(0.5 * dtau * U);
  return std::log1p(m + std::sqrt(m * (m + 2.0)));
}

hfqmc_status validate(const hfqmc_problem& p, int idx) {
  if (p.L < 1 || p.L > kMaxL) return fail(HFQMC_EINVAL, "problem %d: L=%d outside [1,%d]", idx, p.L, kMaxL);
  if (!(p.beta > 0) || !std::isfinite(p.beta)) return fail(HFQMC_EINVAL, "problem %d: beta must be > 0", idx);
  if (!(p.U >= 0) || !std::isfinite(p.U)) return fail(HFQMC_EINVAL, "problem %d: U must be >= 0", idx);
  if (p.n_bins < 2) return fail(HFQMC_EINVAL, "problem %d: n_bins must be >= 2", idx);
  if (p.n_measure < p.n_bins) return fail(HFQMC_EINVAL, "problem %d: n_measure < n_bins", idx);
  if (p.n_warmup < 0) return fail(HFQMC_EINVAL, "problem %d: n_warmup < 0", idx);
  if (p.recompute_every < 1) return fail(HFQMC_EINVAL, "problem %d: recompute_every < 1", idx);
  if (p.delay < 0) return fail(HFQMC_EINVAL, "problem %d: delay < 0", idx);
  for (int s = 0; s < 2; ++s) {
    if (!p.weiss[s]) return fail(HFQMC_EINVAL, "problem %d: weiss[%d] is NULL", idx, s);
    for (int k = 0; k < p.L; ++k)
      if (!std::isfinite(p.weiss[s][k])) return fail(HFQMC_EINVAL, "problem %d: weiss[%d][%d] not finite", idx, s, k);
    if (!(p.weiss[s][0] > 0.0 && p.weiss[s][0] < 1.0))
      return fail(HFQMC_EINVAL, "problem %d: weiss[%d](0+) outside (0,1)", idx, s);
  }
  if (p.init_fields)
    for (int k = 0; k < p.L; ++k)
      if (p.init_fields[k] != 1 && p.init_fields[k] != -1)
        return fail(HFQMC_EINVAL, "problem %d: init_fields[%d] not +-1", idx, k);
  return HFQMC_OK;
}

void fill_constants(ImpDesc& d, const hfqmc_problem& p) {
  const double dtau = p.beta / p.L;
  const double lam = coupling(dtau, p.U);
  d.L = p.L;
  d.lam = lam;
  d.dflip_p = std::expm1(-2.0 * lam);
  d.dflip_m = std::expm1(2.0 * lam);
  d.dset_p = std::expm1(lam);
  d.dset_m = std::expm1(-lam);
  d.n_bins = p.n_bins;
  d.recompute_every = p.recompute_every;
  d.n_warmup = p.n_warmup;
  d.n_measure = p.n_measure;
  d.sweep_begin = 0;
  d.sweep_end = p.n_warmup + p.n_measure;
  d.rng_offset = p.sweep_offset;
  d.seed = p.seed;
  d.site = p.site_id;
  d.delay = p.delay == 0 ? 1 : p.delay;
}

// Bin counts, means and errors from per-bin sums.
void finalise(const hfqmc_problem& p, const double* sums, const ImpStatus& st, const int8_t* fields,
              hfqmc_result& r) {
  const int L = p.L, NV = n_values(L), nb = p.n_bins;
  const int64_t nm = p.n_measure;
  std::vector<int64_t> cnt(nb, 0);
  for (int64_t m = 0; m < nm; ++m) cnt[(m * nb) / nm]++;
  std::vector<double> mean(NV, 0.0), err(NV, 0.0), bm((size_t)nb * NV);
  for (int b = 0; b < nb; ++b)
    for (int v = 0; v < NV; ++v) bm[(size_t)b * NV + v] = sums[(size_t)b * NV + v] / (double)cnt[b];
  for (int v = 0; v < NV; ++v) {
    double s = 0;
    for (int b = 0; b < nb; ++b) s += bm[(size_t)b * NV + v];
    mean[v] = s / nb;
    double ss = 0;
    for (int b = 0; b < nb; ++b) {
      const double dv = bm[(size_t)b * NV + v] - mean[v];
      ss += dv * dv;
    }
    err[v] = std::sqrt(ss / (nb - 1)) / std::sqrt((double)nb);
  }
  for (int s = 0; s < 2; ++s) {
    if (r.g[s]) std::memcpy(r.g[s], &mean[s * (L + 1)], sizeof(double) * (L + 1));
    if (r.g_err[s]) std::memcpy(r.g_err[s], &err[s * (L + 1)], sizeof(double) * (L + 1));
  }
  if (r.bins) std::memcpy(r.bins, bm.data(), sizeof(double) * bm.size());
  if (r.final_fields && fields) std::memcpy(r.final_fields, fields, L);
  r.n[0] = mean[2 * L + 2];
  r.n[1] = mean[2 * L + 3];
  r.docc = mean[2 * L + 4];
  r.n_err[0] = err[2 * L + 2];
  r.n_err[1] = err[2 * L + 3];
  r.docc_err = err[2 * L + 4];
  r.proposals = st.proposals;
  r.accepts = st.accepts;
  r.nonpositive = st.nonpositive;
  r.accept_rate = st.proposals ? (double)st.accepts / (double)st.proposals : 0.0;
  r.max_drift = st.max_drift;
  bool finite = std::isfinite(r.n[0]) && std::isfinite(r.n[1]) && std::isfinite(r.docc);
  r.status = (st.error || !finite) ? HFQMC_ENUMERIC : HFQMC_OK;
}

// State area -> row-major L x L.  Thread t = 64 * wave + lane of the kernel
// owns RT*NT*4 consecutive doubles: tile (rt, tj), register r holds element
// row (wr*RT + rt)*16 + 4*(lane/16) + r, column tj*16 + lane%16, where wave
// = spin*WPS + wr.
void tiles_to_rowmajor(const double* st, int L, int LT, int RT, int spin, double* out) {
  const int NT = LT / 16, WPS = NT / RT;
  const size_t per_lane = (size_t)RT * NT * 4;
  for (int wr = 0; wr < WPS; ++wr)
    for (int lane = 0; lane < 64; ++lane) {
      const double* p = st + ((size_t)(spin * WPS + wr) * 64 + lane) * per_lane;
      for (int rt = 0; rt < RT; ++rt)
        for (int tj = 0; tj < NT; ++tj)
          for (int r = 0; r < 4; ++r) {
            const int i = (wr * RT + rt) * 16 + 4 * (lane / 16) + r, j = tj * 16 + lane % 16;
            if (i < L && j < L) out[(size_t)i * L + j] = p[(rt * NT + tj) * 4 + r];
          }
    }
}

struct Group {
  const KernelInfo* k;
  int first, count, grid;
};

// Workspace layout of one batch.
struct Layout {
  size_t descs, order, queues, weiss, fields, status, bins, state, total;
  std::vector<size_t> w_off, f_off, b_off, s_off;
};

Layout plan_layout(const hfqmc_problem* p, int n) {
  Layout lo;
  size_t off = 0;
  lo.descs = off;
  off = align_up(off + sizeof(ImpDesc) * n, 256);
  lo.order = off;
  off = align_up(off + sizeof(int32_t) * n, 256);
  lo.queues = off;
  off = align_up(off + sizeof(int32_t) * 64, 256);
  lo.weiss = off;
  lo.w_off.resize(n);
  for (int i = 0; i < n; ++i) {
    lo.w_off[i] = off;
    off += sizeof(double) * 2 * p[i].L;
  }
  off = align_up(off, 256);
  lo.fields = off;
  lo.f_off.resize(n);
  for (int i = 0; i < n; ++i) {
    lo.f_off[i] = off;
    off += align_up(p[i].L, 8);
  }
  off = align_up(off, 256);
  lo.status = off;
  off = align_up(off + sizeof(ImpStatus) * n, 256);
  lo.bins = off;
  lo.b_off.resize(n);
  for (int i = 0; i < n; ++i) {
    lo.b_off[i] = off;
    off += sizeof(double) * (size_t)p[i].n_bins * n_values(p[i].L);
  }
  off = align_up(off, 256);
  lo.state = off;
  lo.s_off.resize(n);
  for (int i = 0; i < n; ++i) {
    lo.s_off[i] = off;
    const size_t LT = padded_L(p[i].L);
    off += sizeof(double) * 2 * LT * LT;
  }
  lo.total = align_up(off, 256);
  return lo;
}

struct PoolBlock {
  size_t off, bytes;
};

}  // namespace

struct hfqmc_site {
  int L, LT, RT, n_bins;
  size_t off, bytes;  // pool block
  size_t o_desc, o_weiss, o_fields, o_bins, o_status, o_state, o_force;
  bool defined = false, has_state = false;
  hfqmc_problem prob{};
};

struct hfqmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hfqmc_precision prec = HFQMC_FP64;
  int n_cu = 0;
  std::mutex mu;
  // staged batch
  bool staged = false;
  bool fields_given = false;
  uint8_t* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<hfqmc_problem> probs;
  std::vector<Group> groups;
  Layout lo;
  std::vector<uint8_t> host_in;   // image of descs..fields
  std::vector<uint8_t> host_out;  // image of fields..bins end
  std::vector<hipEvent_t> ev;
  int last_launches = 0;
  // pool
  uint8_t* pool = nullptr;
  size_t pool_bytes = 0;
  std::vector<PoolBlock> free_list;
  std::vector<hfqmc_site*> sites;
  std::string err;
};

namespace {

hfqmc_status set_device(hfqmc_ctx* c) {
  HIP_TRY(hipSetDevice(c->device));
  return HFQMC_OK;
}

hfqmc_status ensure_events(hfqmc_ctx* c, size_t n) {
  while (c->ev.size() < n) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    c->ev.push_back(e);
  }
  return HFQMC_OK;
}

hfqmc_status pool_alloc(hfqmc_ctx* c, size_t bytes, size_t* off) {
  bytes = align_up(bytes, 256);
  for (size_t i = 0; i < c->free_list.size(); ++i) {
    PoolBlock& b = c->free_list[i];
    if (b.bytes >= bytes) {
      *off = b.off;
      b.off += bytes;
      b.bytes -= bytes;
      if (b.bytes == 0) c->free_list.erase(c->free_list.begin() + i);
      return HFQMC_OK;
    }
  }
  return fail(HFQMC_ENOMEM, "pool exhausted: need %zu bytes", bytes);
}

void pool_free(hfqmc_ctx* c, size_t off, size_t bytes) {
  bytes = align_up(bytes, 256);
  c->free_list.push_back({off, bytes});
  std::sort(c->free_list.begin(), c->free_list.end(), [](const PoolBlock& a, const PoolBlock& b) { return a.off < b.off; });
  std::vector<PoolBlock> merged;
  for (const auto& b : c->free_list) {
    if (!merged.empty() && merged.back().off + merged.back().bytes == b.off)
      merged.back().bytes += b.bytes;
    else
      merged.push_back(b);
  }
  c->free_list.swap(merged);
}

size_t site_layout(hfqmc_site* s) {
  size_t off = 0;
  s->o_desc = off;
  off = align_up(off + sizeof(ImpDesc), 256);
  s->o_weiss = off;
  off = align_up(off + sizeof(double) * 2 * s->L, 256);
  s->o_fields = off;
  off = align_up(off + s->L, 256);
  s->o_status = off;
  off = align_up(off + sizeof(ImpStatus), 256);
  s->o_bins = off;
  off = align_up(off + sizeof(double) * (size_t)s->n_bins * n_values(s->L), 256);
  s->o_state = off;
  off = align_up(off + sizeof(double) * 2 * (size_t)s->LT * s->LT, 256);
  s->o_force = off;
  off = align_up(off + 1024 * (sizeof(int32_t) + sizeof(double)), 256);
  // queue counter + order entry
  off = align_up(off + 256, 256);
  return off;
}

// Launch one work item on a site (blocking).
hfqmc_status site_launch(hfqmc_ctx* c, hfqmc_site* s, ImpDesc d) {
  uint8_t* base = c->pool + s->off;
  d.off_weiss = (int64_t)s->o_weiss;
  d.off_fields = (int64_t)s->o_fields;
  d.off_bins = (int64_t)s->o_bins;
  d.off_status = (int64_t)s->o_status;
  d.off_state = (int64_t)s->o_state;
  d.off_force = (int64_t)s->o_force;
  d.LT = s->LT;
  const KernelInfo* k = find_kernel(s->LT, s->RT, 0);
  if (!k) return fail(HFQMC_EINVAL, "no kernel for LT=%d RT=%d", s->LT, s->RT);
  const size_t qoff = s->o_force + align_up(1024 * (sizeof(int32_t) + sizeof(double)), 256);
  struct {
    int32_t queue, order;
  } qo = {0, 0};
  HIP_TRY(hipMemcpyAsync(base + s->o_desc, &d, sizeof d, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(base + qoff, &qo, sizeof qo, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(launch_sweep(k, 1, c->stream, reinterpret_cast<const ImpDesc*>(base + s->o_desc),
                       reinterpret_cast<const int32_t*>(base + qoff + 4), 1, reinterpret_cast<int*>(base + qoff),
                       base));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return HFQMC_OK;
}

}  // namespace

extern "C" {

hfqmc_status hfqmc_lambda(double dtau, double U, double* lambda_out) {
  if (!lambda_out || !(dtau > 0) || !(U >= 0) || !std::isfinite(dtau) || !std::isfinite(U))
    return fail(HFQMC_EINVAL, "hfqmc_lambda: need dtau > 0, U >= 0");
  *lambda_out = coupling(dtau, U);
  return HFQMC_OK;
}

hfqmc_status hfqmc_create(int device, void* hip_stream, hfqmc_precision precision, const char* tune_cache,
                          hfqmc_ctx** out) {
  (void)tune_cache;
  if (!out) return fail(HFQMC_EINVAL, "hfqmc_create: out is NULL");
  if (precision != HFQMC_FP64 && precision != HFQMC_MIXED) return fail(HFQMC_EINVAL, "bad precision");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(HFQMC_EINVAL, "device %d outside [0,%d)", device, ndev);
  hfqmc_ctx* c = new (std::nothrow) hfqmc_ctx;
  if (!c) return fail(HFQMC_ENOMEM, "out of host memory");
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->prec = precision;
  hipDeviceProp_t prop;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete c;
    return fail(HFQMC_EDEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    delete c;
    return fail(HFQMC_EDEVICE, "device %d is %s; this library is built for gfx950 only", device, prop.gcnArchName);
  }
  c->n_cu = prop.multiProcessorCount;
  *out = c;
  return HFQMC_OK;
}

void hfqmc_destroy(hfqmc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (auto e : c->ev) (void)hipEventDestroy(e);
  for (auto s : c->sites) delete s;
  delete c;
}

const char* hfqmc_last_error(const hfqmc_ctx*) { return t_err.c_str(); }

hfqmc_status hfqmc_workspace_size(hfqmc_ctx* c, const hfqmc_problem* p, int32_t n, size_t* bytes) {
  if (!c || !bytes || n < 0 || (n > 0 && !p)) return fail(HFQMC_EINVAL, "hfqmc_workspace_size: bad arguments");
  for (int i = 0; i < n; ++i) {
    hfqmc_status s = validate(p[i], i);
    if (s) return s;
  }
  *bytes = plan_layout(p, n).total;
  return HFQMC_OK;
}

hfqmc_status hfqmc_stage(hfqmc_ctx* c, const hfqmc_problem* p, int32_t n, void* d_ws, size_t ws_bytes) {
  if (!c || n < 1 || !p || !d_ws) return fail(HFQMC_EINVAL, "hfqmc_stage: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  for (int i = 0; i < n; ++i) {
    hfqmc_status s = validate(p[i], i);
    if (s) return s;
  }
  Layout lo = plan_layout(p, n);
  if (ws_bytes < lo.total) return fail(HFQMC_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, lo.total);
  if (hfqmc_status s = set_device(c)) return s;

  // group items by kernel class (padded L, update kind); inside a class order
  // items by descending work
  std::vector<int> idx(n), kind(n);
  for (int i = 0; i < n; ++i) {
    idx[i] = i;
    kind[i] = update_kind(p[i], c->prec);
    if (kind[i] && !find_kernel(padded_L(p[i].L), choose_rt(padded_L(p[i].L), kind[i]), kind[i]))
      return fail(HFQMC_EINVAL, "problem %d: no delayed-update kernel for L=%d", i, p[i].L);
    if (p[i].delay > 32) return fail(HFQMC_EINVAL, "problem %d: delay %d > 32", i, p[i].delay);
  }
  auto cost = [&](int i) { return (double)(p[i].n_warmup + p[i].n_measure) * p[i].L * p[i].L; };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    const int la = padded_L(p[a].L), lb = padded_L(p[b].L);
    if (la != lb) return la > lb;
    if (kind[a] != kind[b]) return kind[a] < kind[b];
    return cost(a) > cost(b);
  });
  std::vector<Group> groups;
  for (int k = 0; k < n;) {
    const int LT = padded_L(p[idx[k]].L), DK = kind[idx[k]];
    int e = k;
    while (e < n && padded_L(p[idx[e]].L) == LT && kind[idx[e]] == DK) ++e;
    const KernelInfo* ki = find_kernel(LT, choose_rt(LT, DK), DK);
    if (!ki) return fail(HFQMC_EINVAL, "no kernel for padded L=%d", LT);
    int bpc = 0;
    HIP_TRY(kernel_occupancy(ki, &bpc));
    if (bpc < 1) return fail(HFQMC_EDEVICE, "kernel for L=%d does not fit on a CU", LT);
    const int grid = std::min(e - k, bpc * c->n_cu);
    groups.push_back({ki, k, e - k, grid});
    k = e;
  }
  if (groups.size() > 64) return fail(HFQMC_EINVAL, "too many kernel classes");

  // host image of the input region [descs, fields end)
  std::vector<uint8_t> img(lo.status, 0);
  ImpDesc* descs = reinterpret_cast<ImpDesc*>(img.data() + lo.descs);
  int32_t* order = reinterpret_cast<int32_t*>(img.data() + lo.order);
  for (int i = 0; i < n; ++i) {
    ImpDesc d{};
    fill_constants(d, p[i]);
    d.LT = padded_L(p[i].L);
    d.op = OP_SWEEPS;
    d.flags = F_ZERO_ACC | (p[i].init_fields ? F_FIELDS_GIVEN : 0) | F_SAVE;
    d.off_weiss = (int64_t)lo.w_off[i];
    d.off_fields = (int64_t)lo.f_off[i];
    d.off_bins = (int64_t)lo.b_off[i];
    d.off_status = (int64_t)(lo.status + sizeof(ImpStatus) * i);
    d.off_state = (int64_t)lo.s_off[i];
    d.off_force = 0;
    descs[i] = d;
    std::memcpy(img.data() + lo.w_off[i], p[i].weiss[0], sizeof(double) * p[i].L);
    std::memcpy(img.data() + lo.w_off[i] + sizeof(double) * p[i].L, p[i].weiss[1], sizeof(double) * p[i].L);
    if (p[i].init_fields) std::memcpy(img.data() + lo.f_off[i], p[i].init_fields, p[i].L);
  }
  for (int i = 0; i < n; ++i) order[i] = idx[i];
  c->ws = reinterpret_cast<uint8_t*>(d_ws);
  c->ws_bytes = ws_bytes;
  HIP_TRY(hipMemcpyAsync(c->ws, img.data(), img.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->probs.assign(p, p + n);
  c->groups = groups;
  c->lo = lo;
  c->host_in.swap(img);
  c->fields_given = false;
  for (int i = 0; i < n; ++i) c->fields_given |= p[i].init_fields != nullptr;
  c->staged = true;
  return HFQMC_OK;
}

hfqmc_status hfqmc_run(hfqmc_ctx* c) {
  if (!c || !c->staged) return fail(HFQMC_EINVAL, "hfqmc_run: nothing staged");
  std::lock_guard<std::mutex> g(c->mu);
  if (hfqmc_status s = set_device(c)) return s;
  // fields are inputs when given: restore them (a previous run overwrote them)
  if (c->fields_given) {
    const size_t fbytes = c->lo.status - c->lo.fields;
    HIP_TRY(hipMemcpyAsync(c->ws + c->lo.fields, c->host_in.data() + c->lo.fields, fbytes, hipMemcpyHostToDevice,
                           c->stream));
  }
  HIP_TRY(launch_zero(c->ws + c->lo.queues, sizeof(int32_t) * 64, c->stream));
  if (hfqmc_status s = ensure_events(c, 2 * c->groups.size())) return s;
  const ImpDesc* descs = reinterpret_cast<const ImpDesc*>(c->ws + c->lo.descs);
  const int32_t* order = reinterpret_cast<const int32_t*>(c->ws + c->lo.order);
  int* queues = reinterpret_cast<int*>(c->ws + c->lo.queues);
  for (size_t gi = 0; gi < c->groups.size(); ++gi) {
    const Group& gr = c->groups[gi];
    HIP_TRY(hipEventRecord(c->ev[2 * gi], c->stream));
    HIP_TRY(launch_sweep(gr.k, gr.grid, c->stream, descs, order + gr.first, gr.count, queues + gi, c->ws));
    HIP_TRY(hipEventRecord(c->ev[2 * gi + 1], c->stream));
  }
  c->last_launches = (int)c->groups.size();
  return HFQMC_OK;
}

hfqmc_status hfqmc_last_run_ms(hfqmc_ctx* c, double* ms, int32_t* n_launches) {
  if (!c || !ms) return fail(HFQMC_EINVAL, "hfqmc_last_run_ms: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (c->last_launches == 0) return fail(HFQMC_EINVAL, "no run recorded");
  HIP_TRY(hipEventSynchronize(c->ev[2 * c->last_launches - 1]));
  float t = 0.f;
  HIP_TRY(hipEventElapsedTime(&t, c->ev[0], c->ev[2 * c->last_launches - 1]));
  *ms = t;
  if (n_launches) *n_launches = c->last_launches;
  return HFQMC_OK;
}

hfqmc_status hfqmc_collect(hfqmc_ctx* c, hfqmc_result* out) {
  if (!c || !c->staged || !out) return fail(HFQMC_EINVAL, "hfqmc_collect: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (hfqmc_status s = set_device(c)) return s;
  const size_t lo_off = c->lo.fields, hi_off = c->lo.state;
  c->host_out.resize(hi_off - lo_off);
  HIP_TRY(hipMemcpyAsync(c->host_out.data(), c->ws + lo_off, hi_off - lo_off, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  hfqmc_status worst = HFQMC_OK;
  for (size_t i = 0; i < c->probs.size(); ++i) {
    const hfqmc_problem& p = c->probs[i];
    const double* sums = reinterpret_cast<const double*>(c->host_out.data() + (c->lo.b_off[i] - lo_off));
    const ImpStatus* st =
        reinterpret_cast<const ImpStatus*>(c->host_out.data() + (c->lo.status - lo_off) + sizeof(ImpStatus) * i);
    const int8_t* fields = reinterpret_cast<const int8_t*>(c->host_out.data() + (c->lo.f_off[i] - lo_off));
    finalise(p, sums, *st, fields, out[i]);
    if (out[i].status != HFQMC_OK) worst = (hfqmc_status)out[i].status;
  }
  if (worst != HFQMC_OK) return fail(worst, "non-finite ratio or Green function in at least one impurity");
  return HFQMC_OK;
}

hfqmc_status hfqmc_solve(hfqmc_ctx* c, const hfqmc_problem* p, int32_t n, void* d_ws, size_t ws_bytes,
                         hfqmc_result* out) {
  if (!out) return fail(HFQMC_EINVAL, "hfqmc_solve: out is NULL");
  hfqmc_status s = hfqmc_stage(c, p, n, d_ws, ws_bytes);
  if (s) return s;
  s = hfqmc_run(c);
  if (s) return s;
  return hfqmc_collect(c, out);
}

// ---------------------------------------------------------------- sites

hfqmc_status hfqmc_attach_pool(hfqmc_ctx* c, void* d_pool, size_t bytes) {
  if (!c || !d_pool || bytes < 4096) return fail(HFQMC_EINVAL, "hfqmc_attach_pool: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!c->sites.empty()) return fail(HFQMC_EINVAL, "hfqmc_attach_pool: sites still open");
  c->pool = reinterpret_cast<uint8_t*>(d_pool);
  c->pool_bytes = bytes;
  c->free_list.assign(1, PoolBlock{0, bytes / 256 * 256});
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_bytes(int32_t L, int32_t n_bins, size_t* bytes) {
  if (L < 1 || L > kMaxL || n_bins < 2 || !bytes) return fail(HFQMC_EINVAL, "hfqmc_site_bytes: bad arguments");
  hfqmc_site s;
  s.L = L;
  s.LT = padded_L(L);
  s.n_bins = n_bins;
  *bytes = site_layout(&s);
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_open(hfqmc_ctx* c, int32_t L, int32_t n_bins, hfqmc_site** out) {
  if (!c || !out || L < 1 || L > kMaxL || n_bins < 2) return fail(HFQMC_EINVAL, "hfqmc_site_open: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!c->pool) return fail(HFQMC_EINVAL, "hfqmc_site_open: no pool attached");
  hfqmc_site* s = new (std::nothrow) hfqmc_site;
  if (!s) return fail(HFQMC_ENOMEM, "out of host memory");
  s->L = L;
  s->LT = padded_L(L);
  s->RT = choose_rt(s->LT);
  s->n_bins = n_bins;
  s->bytes = site_layout(s);
  if (hfqmc_status st = pool_alloc(c, s->bytes, &s->off)) {
    delete s;
    return st;
  }
  c->sites.push_back(s);
  *out = s;
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_close(hfqmc_ctx* c, hfqmc_site* s) {
  if (!c || !s) return fail(HFQMC_EINVAL, "hfqmc_site_close: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  auto it = std::find(c->sites.begin(), c->sites.end(), s);
  if (it == c->sites.end()) return fail(HFQMC_ENOTFOUND, "unknown site");
  pool_free(c, s->off, s->bytes);
  c->sites.erase(it);
  delete s;
  return HFQMC_OK;
}

static bool site_known(hfqmc_ctx* c, hfqmc_site* s) {
  return std::find(c->sites.begin(), c->sites.end(), s) != c->sites.end();
}

hfqmc_status hfqmc_site_define(hfqmc_ctx* c, hfqmc_site* s, const hfqmc_problem* p) {
  if (!c || !s || !p) return fail(HFQMC_EINVAL, "hfqmc_site_define: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!site_known(c, s)) return fail(HFQMC_ENOTFOUND, "unknown site");
  if (p->L != s->L || p->n_bins != s->n_bins) return fail(HFQMC_EINVAL, "problem L/n_bins differ from the site's");
  if (hfqmc_status st = validate(*p, 0)) return st;
  if (hfqmc_status st = set_device(c)) return st;
  uint8_t* base = c->pool + s->off;
  HIP_TRY(hipMemcpyAsync(base + s->o_weiss, p->weiss[0], sizeof(double) * s->L, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(base + s->o_weiss + sizeof(double) * s->L, p->weiss[1], sizeof(double) * s->L,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  s->prob = *p;
  s->prob.weiss[0] = s->prob.weiss[1] = nullptr;
  s->prob.init_fields = nullptr;
  s->defined = true;
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_set_fields(hfqmc_ctx* c, hfqmc_site* s, const int8_t* fields) {
  if (!c || !s || !fields) return fail(HFQMC_EINVAL, "hfqmc_site_set_fields: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!site_known(c, s)) return fail(HFQMC_ENOTFOUND, "unknown site");
  if (!s->defined) return fail(HFQMC_EINVAL, "site has no problem (call hfqmc_site_define)");
  for (int k = 0; k < s->L; ++k)
    if (fields[k] != 1 && fields[k] != -1) return fail(HFQMC_EINVAL, "fields[%d] not +-1", k);
  if (hfqmc_status st = set_device(c)) return st;
  HIP_TRY(hipMemcpyAsync(c->pool + s->off + s->o_fields, fields, s->L, hipMemcpyHostToDevice, c->stream));
  ImpDesc d{};
  fill_constants(d, s->prob);
  d.op = OP_FORCE;
  d.n_force = 0;
  d.flags = F_FIELDS_GIVEN | F_SAVE | F_ZERO_ACC;
  if (hfqmc_status st = site_launch(c, s, d)) return st;
  s->has_state = true;
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_force_flips(hfqmc_ctx* c, hfqmc_site* s, const int32_t* slices, int32_t n, double* ratios) {
  if (!c || !s || n < 0 || (n > 0 && !slices)) return fail(HFQMC_EINVAL, "hfqmc_site_force_flips: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!site_known(c, s)) return fail(HFQMC_ENOTFOUND, "unknown site");
  if (!s->has_state) return fail(HFQMC_EINVAL, "site has no state (call hfqmc_site_set_fields)");
  for (int k = 0; k < n; ++k)
    if (slices[k] < 0 || slices[k] >= s->L) return fail(HFQMC_EINVAL, "slice %d outside [0,%d)", slices[k], s->L);
  if (hfqmc_status st = set_device(c)) return st;
  uint8_t* base = c->pool + s->off;
  for (int k0 = 0; k0 < n; k0 += 1024) {
    const int m = std::min(1024, n - k0);
    HIP_TRY(hipMemcpyAsync(base + s->o_force, slices + k0, sizeof(int32_t) * m, hipMemcpyHostToDevice, c->stream));
    ImpDesc d{};
    fill_constants(d, s->prob);
    d.op = OP_FORCE;
    d.n_force = m;
    d.flags = F_RESUME | F_SAVE;
    if (hfqmc_status st = site_launch(c, s, d)) return st;
    if (ratios) {
      HIP_TRY(hipMemcpy(ratios + k0, base + s->o_force + 4 * ((m + 1) & ~1), sizeof(double) * m,
                        hipMemcpyDeviceToHost));
    }
  }
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_recompute(hfqmc_ctx* c, hfqmc_site* s, double* drift) {
  if (!c || !s) return fail(HFQMC_EINVAL, "hfqmc_site_recompute: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!site_known(c, s)) return fail(HFQMC_ENOTFOUND, "unknown site");
  if (!s->has_state) return fail(HFQMC_EINVAL, "site has no state");
  if (hfqmc_status st = set_device(c)) return st;
  ImpDesc d{};
  fill_constants(d, s->prob);
  d.op = OP_RECOMPUTE;
  d.flags = F_RESUME | F_SAVE | F_ZERO_ACC;
  if (hfqmc_status st = site_launch(c, s, d)) return st;
  if (drift) {
    ImpStatus st;
    HIP_TRY(hipMemcpy(&st, c->pool + s->off + s->o_status, sizeof st, hipMemcpyDeviceToHost));
    *drift = st.max_drift;
  }
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_get_green(hfqmc_ctx* c, hfqmc_site* s, int32_t spin, double* out) {
  if (!c || !s || !out || (spin != 0 && spin != 1)) return fail(HFQMC_EINVAL, "hfqmc_site_get_green: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!site_known(c, s)) return fail(HFQMC_ENOTFOUND, "unknown site");
  if (!s->has_state) return fail(HFQMC_EINVAL, "site has no state");
  if (hfqmc_status st = set_device(c)) return st;
  std::vector<double> st((size_t)2 * s->LT * s->LT);
  HIP_TRY(hipMemcpyAsync(st.data(), c->pool + s->off + s->o_state, sizeof(double) * st.size(), hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  tiles_to_rowmajor(st.data(), s->L, s->LT, s->RT, spin, out);
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_get_fields(hfqmc_ctx* c, hfqmc_site* s, int8_t* fields) {
  if (!c || !s || !fields) return fail(HFQMC_EINVAL, "hfqmc_site_get_fields: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!site_known(c, s)) return fail(HFQMC_ENOTFOUND, "unknown site");
  if (!s->has_state) return fail(HFQMC_EINVAL, "site has no state");
  if (hfqmc_status st = set_device(c)) return st;
  HIP_TRY(hipMemcpyAsync(fields, c->pool + s->off + s->o_fields, s->L, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return HFQMC_OK;
}

}  // extern "C"
