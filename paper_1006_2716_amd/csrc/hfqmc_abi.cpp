// hfqmc_abi.cpp -- host side of the C ABI declared in include/hfqmc.h.
//
// Validates problems, computes the HS coupling, plans the batch (one kernel
// class per padded slice count and update kind), lays out the caller's
// workspace, launches the gfx950 kernels (classes concurrently on forked
// streams, optionally replayed from a captured hipGraph), autotunes the
// kernel shape per class, finalises bin statistics, and runs the serving
// engine: a host thread that admits impurity-solve requests on
// device-resident sites and advances them in short launches (continuous
// batching).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "hfqmc.h"
#include "hfqmc_internal.h"
#include "hfqmc_lattice.h"

namespace hfqmc {
struct KernelInfo;
const KernelInfo* find_kernel(int LT, int RT, int DK);
int kernel_variants(int LT, int DK, int* rt_out, int max);
int kernel_threads(const KernelInfo* k);
size_t kernel_lds(const KernelInfo* k);
hipError_t kernel_occupancy(const KernelInfo* k, int* blocks_per_cu);
hipError_t launch_sweep(const KernelInfo* k, int grid, hipStream_t st, const ImpDesc* descs, const int32_t* order,
                        int n_items, int* queue, uint8_t* ws);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
size_t lattice_work_bytes(int layer, int n_layers, int n_freq);
hipError_t launch_lattice_green(const LatDesc& d, hipStream_t st);
hipError_t launch_weiss(const WeissDesc& d, hipStream_t st);
hipError_t launch_sigma(const SigmaDesc& d, hipStream_t st);
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

#define TRY(expr)                        \
  do {                                   \
    hfqmc_status s_ = (expr);            \
    if (s_ != HFQMC_OK) return s_;       \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// The device array behind hfqmc_solve_static, and its address on each device
// (resolved once per device by hfqmc_create with that device current: in
// host code the array's name is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[HFQMC_STATIC_BYTES];

namespace {

hfqmc_status scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(HFQMC_EINVAL, "device %d outside [0,%d)", device, kMaxDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return HFQMC_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return fail(HFQMC_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_scratch_ptr[device] = p;
  return HFQMC_OK;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

int padded_L(int L) { return (L + 15) / 16 * 16; }

constexpr int kMaxDelay = 32;    // panel capacity of the delayed-update kernels
// Default drift limit of HFQMC_MIXED contexts (fp32 products in the window
// flush drift by ~1e-4 per sweep at U up to 12): at or below the statistical
// errors of the estimators over runs of thousands of sweeps.
constexpr double kMixedDriftLimit = 1e-3;
constexpr int kAuxStreams = 3;   // extra streams for concurrent kernel classes
constexpr int kSrvStreams = 6;   // serving launch streams
constexpr int kMaxChains = 64;   // independent chains per problem

// Kernel shape of one class: tile-rows per wave, update kind (0 plain
// rank-one, 1 delayed fp64, 2 delayed mixed, 3 window updates, 4 window
// updates with fp32 products), delay depth (0 for window updates) and the
// kernel's padded slice count.
struct Plan {
  int rt = 1, dk = 0, k = 1, LT = 16;
};

constexpr int kDkWindow = 3, kDkWindowMixed = 4;
inline bool is_window(int dk) { return dk == kDkWindow || dk == kDkWindowMixed; }

// Padded slice count of the window kernel serving L <= 128: the next
// multiple of 16 up to 96, then 128 (no 112-slice window kernel is built:
// seven tile columns leave one tile-row per wave, fourteen waves whose
// 128-register budget spills, or seven, 392 registers of tiles).
int window_LT(int L) {
  if (L <= 96) return (L + 15) / 16 * 16;
  return 128;
}

// Padded slice count of the kernel of update kind dk for L slices.
int kernel_LT(int L, int dk) { return is_window(dk) && L <= kMaxRegisterL ? window_LT(L) : (L + 15) / 16 * 16; }

// Padded slice counts at which the untuned default is the window kernel
// (elsewhere the rank-one kernel, measured faster there on MI355X).
bool window_default(int LT) {
  // 512 impurities of the chain workload: 159 against 228 ms at 80 slices,
  // 209 against 284 ms at 96, 335 against 504 ms at 128; at 32-64 slices
  // the rank-one kernels are 4-25 % faster (48: 59 against 65 ms, 64: 75
  // against 79)
  return LT >= 80;
}

// Untuned tile-rows per wave of the window kernels, each the measured best
// on 512 impurities of the chain workload at that L: 48 slices 3 (65 ms),
// 64 slices 2 (79 ms; 109 with one), 80 slices 5 (159 against 167 with one;
// 393 against 466 ms on the 1281 slab sites, where five tile-rows per wave
// put two impurities on a CU), 96 slices 1 (209 against 245 with 3), 128
// slices 2 (335 against 505 with 4).  With fp32 flush products one tile-row
// per wave at 80 slices (the slab: 3.4 s against 5.1 s with five, whose
// registers spill with the fp32 conversions).
int default_rt_window(int LT, bool mixed) {
  switch (LT) {
    case 48: return 3;
    case 64: return 2;
    case 80: return mixed ? 1 : 5;
    case 128: return 2;
    default: return 1;
  }
}

// Untuned default tile-rows per wave, each the measured best of the rank-one
// kernels on MI355X: 2 at 64 (512 impurities: 76 ms against 103 with 1 and
// 89 with 4) and 128 (323 ms against 1404); one wave per spin at 48 (25-34 %
// faster than three waves per spin on 325-site trapped batches, 3 % slower
// on 100 impurities) and 96 (195 ms against 214 with 1 and 243 with 2, 105
// impurities; 357 against 392 and 449 on 1281); 1 at 32 (two waves per spin
// beat one by 8-10 %) and wherever only that variant exists.
int default_rt(int LT, int dk) {
  if (dk == 0 && (LT == 48 || LT == 96)) return 3;
  if (dk == 0 && (LT == 64 || LT == 128)) return 2;
  if (dk != 0 && LT == 64) return 2;
  return 1;
}

// Bytes of state per impurity: G of both spins, then a second 2 L^2 region
// (the drift snapshot of the device-memory kernel, the parked bin sums of G
// of the register kernels), then 3 x 64 parked per-lane sums.
size_t state_bytes(int L) {
  // large enough for every kernel that can run L slices (window kernels may
  // pad further than the next multiple of 16)
  const size_t LT = (size_t)(L <= kMaxRegisterL ? window_LT(L) : (L + 15) / 16 * 16);
  return sizeof(double) * (4 * LT * LT + 256);
}

// HS coupling from cosh(lambda) = exp(dtau U / 2), written as
// acosh(1 + m) = log1p(m + sqrt(m (m + 2))) with m = expm1(dtau U / 2).
double coupling(double dtau, double U) {
  const double m = std::expm1(0.5 * dtau * U);
  return std::log1p(m + std::sqrt(m * (m + 2.0)));
}

// Chains of one problem (0 and 1 both mean one) and the measured sweeps of
// chain j: an equal share, the first n_measure % n_chains chains one more.
int chains_of(const hfqmc_problem& p) { return p.n_chains > 1 ? p.n_chains : 1; }
int64_t chain_measure(const hfqmc_problem& p, int j) {
  const int nc = chains_of(p);
  return p.n_measure / nc + (j < p.n_measure % nc ? 1 : 0);
}

hfqmc_status validate(const hfqmc_problem& p, int idx) {
  if (p.L < 1 || p.L > kMaxL) return fail(HFQMC_EINVAL, "problem %d: L=%d outside [1,%d]", idx, p.L, kMaxL);
  if (!(p.beta > 0) || !std::isfinite(p.beta)) return fail(HFQMC_EINVAL, "problem %d: beta must be > 0", idx);
  if (!(p.U >= 0) || !std::isfinite(p.U)) return fail(HFQMC_EINVAL, "problem %d: U must be >= 0", idx);
  if (p.n_bins < 2) return fail(HFQMC_EINVAL, "problem %d: n_bins must be >= 2", idx);
  if (p.n_chains < 0 || p.n_chains > kMaxChains)
    return fail(HFQMC_EINVAL, "problem %d: n_chains outside [0,%d]", idx, kMaxChains);
  if (p.n_measure < (int64_t)chains_of(p) * p.n_bins)
    return fail(HFQMC_EINVAL, "problem %d: n_measure < n_chains * n_bins", idx);
  if (p.n_warmup < 0) return fail(HFQMC_EINVAL, "problem %d: n_warmup < 0", idx);
  if (p.recompute_every < 1) return fail(HFQMC_EINVAL, "problem %d: recompute_every < 1", idx);
  if (p.delay < 0 || p.delay > kMaxDelay) return fail(HFQMC_EINVAL, "problem %d: delay outside [0,%d]", idx, kMaxDelay);
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
  d.delay = 1;
}

// Add the measurement count of each bin of a chain with nm measured sweeps
// (sweep m falls in bin floor(m nb / nm)).
void add_bin_counts(int64_t nm, int nb, int64_t* cnt) {
  for (int64_t m = 0; m < nm; ++m) cnt[(m * nb) / nm]++;
}

// Adds one chain's bin sums and status into the pooled ones.
void pool_chain(int NV, int nb, const double* sums, const ImpStatus& st, double* psums, ImpStatus& pst) {
  for (size_t k = 0; k < (size_t)nb * NV; ++k) psums[k] += sums[k];
  pst.proposals += st.proposals;
  pst.accepts += st.accepts;
  pst.nonpositive += st.nonpositive;
  pst.error |= st.error;
  pst.max_drift = std::max(pst.max_drift, st.max_drift);
  pst.recoveries += st.recoveries;
}

// Bin means and errors from per-bin sums and measurement counts (pooled over
// the chains of the problem).
void finalise(int L, int nb, const double* sums, const int64_t* cnt, const ImpStatus& st, const int8_t* fields,
              hfqmc_result& r) {
  const int NV = n_values(L);
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
  r.recoveries = st.recoveries;
  bool finite = std::isfinite(r.n[0]) && std::isfinite(r.n[1]) && std::isfinite(r.docc);
  r.status = (st.error || !finite) ? HFQMC_ENUMERIC : HFQMC_OK;
}

// State area -> row-major L x L.  Thread t = 64 * wave + lane of the kernel
// owns RT*NT*4 consecutive doubles: tile (rt, tj), register r holds element
// row (wr*RT + rt)*16 + 4*(lane/16) + r, column tj*16 + lane%16, where wave
// = spin*WPS + wr.
void tiles_to_rowmajor(const double* st, int L, int LT, int RT, int spin, double* out) {
  if (RT == 0) {  // global-memory kernel: row-major already
    for (int i = 0; i < L; ++i)
      for (int j = 0; j < L; ++j) out[(size_t)i * L + j] = st[(size_t)spin * LT * LT + (size_t)i * LT + j];
    return;
  }
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
  int LT, rt, dk;
  int first, count, grid;
  int stream = 0;  // index into the pass's streams (0: the context stream)
  bool tuned = false;  // the class an autotuning run times
};

// A batch with every problem split into its chains: item k runs chain
// chain[k] of problem owner[k], with that chain's measured sweeps.
struct Expanded {
  std::vector<hfqmc_problem> items;
  std::vector<int> owner, chain;
};

Expanded expand(const hfqmc_problem* p, int n) {
  Expanded e;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < chains_of(p[i]); ++j) {
      hfqmc_problem q = p[i];
      q.n_measure = chain_measure(p[i], j);
      q.n_chains = 1;
      e.items.push_back(q);
      e.owner.push_back(i);
      e.chain.push_back(j);
    }
  return e;
}

// Workspace layout of one batch.
struct Layout {
  size_t descs, order, queues, weiss, init, fields, status, bins, state, total;
  std::vector<size_t> w_off, i_off, f_off, b_off, s_off;
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
  lo.init = off;
  lo.i_off.resize(n);
  for (int i = 0; i < n; ++i) {
    lo.i_off[i] = off;
    off += align_up(p[i].L, 8);
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
    off += state_bytes(p[i].L);
  }
  lo.total = align_up(off, 256);
  return lo;
}

struct PoolBlock {
  size_t off, bytes;
};

// Autotune cache entry: best shape for one padded slice count.
struct TuneEntry {
  std::string prec;
  int LT, rt, k;
  double rate;
  std::string measured;  // every candidate timed: [rt, k, proposals/s], ...
};

const char* prec_name(hfqmc_precision p) { return p == HFQMC_MIXED ? "mixed" : "fp64"; }

// ---- minimal reader for the cache file this library writes ----
bool json_find_num(const std::string& obj, const char* key, double* v) {
  const std::string k = std::string("\"") + key + "\"";
  size_t pos = obj.find(k);
  if (pos == std::string::npos) return false;
  pos = obj.find(':', pos + k.size());
  if (pos == std::string::npos) return false;
  const char* b = obj.c_str() + pos + 1;
  char* e = nullptr;
  *v = std::strtod(b, &e);
  return e != b;
}

bool json_find_str(const std::string& obj, const char* key, std::string* v) {
  const std::string k = std::string("\"") + key + "\"";
  size_t pos = obj.find(k);
  if (pos == std::string::npos) return false;
  pos = obj.find(':', pos + k.size());
  if (pos == std::string::npos) return false;
  const size_t q0 = obj.find('"', pos + 1);
  if (q0 == std::string::npos) return false;
  const size_t q1 = obj.find('"', q0 + 1);
  if (q1 == std::string::npos) return false;
  *v = obj.substr(q0 + 1, q1 - q0 - 1);
  return true;
}

// Text inside the brackets of array `key` (nested brackets kept).
bool json_find_array(const std::string& obj, const char* key, std::string* v) {
  const std::string k = std::string("\"") + key + "\"";
  size_t pos = obj.find(k);
  if (pos == std::string::npos) return false;
  const size_t b = obj.find('[', pos + k.size());
  if (b == std::string::npos) return false;
  int depth = 0;
  for (size_t i = b; i < obj.size(); ++i) {
    if (obj[i] == '[') ++depth;
    if (obj[i] == ']' && --depth == 0) {
      *v = obj.substr(b + 1, i - b - 1);
      return true;
    }
  }
  return false;
}

std::vector<TuneEntry> read_tune_cache(const std::string& path) {
  std::vector<TuneEntry> out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  std::string arch;
  if (!json_find_str(text, "arch", &arch) || arch != "gfx950") return out;
  size_t pos = text.find("\"entries\"");
  if (pos == std::string::npos) return out;
  pos = text.find('[', pos);
  while (pos != std::string::npos) {
    const size_t b = text.find('{', pos), e = b == std::string::npos ? b : text.find('}', b);
    if (b == std::string::npos || e == std::string::npos) break;
    const std::string obj = text.substr(b, e - b + 1);
    TuneEntry t;
    double LT, rt, k, rate = 0;
    if (json_find_str(obj, "precision", &t.prec) && json_find_num(obj, "L_padded", &LT) &&
        json_find_num(obj, "rt", &rt) && json_find_num(obj, "k", &k)) {
      json_find_num(obj, "proposals_per_s", &rate);
      json_find_array(obj, "measured", &t.measured);
      t.LT = (int)LT;
      t.rt = (int)rt;
      t.k = (int)k;
      t.rate = rate;
      out.push_back(t);
    }
    pos = e + 1;
  }
  return out;
}

bool write_tune_cache(const std::string& path, const std::vector<TuneEntry>& v) {
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\"arch\": \"gfx950\", \"entries\": [\n");
  for (size_t i = 0; i < v.size(); ++i)
    std::fprintf(f,
                 "  {\"precision\": \"%s\", \"L_padded\": %d, \"rt\": %d, \"k\": %d, \"proposals_per_s\": %.6g, "
                 "\"measured\": [%s]}%s\n",
                 v[i].prec.c_str(), v[i].LT, v[i].rt, v[i].k, v[i].rate, v[i].measured.c_str(),
                 i + 1 < v.size() ? "," : "");
  std::fprintf(f, "]}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace

// ------------------------------------------------------------- sites & serving

struct hfqmc_site {
  int L, LT, RT, n_bins;
  int n_chains = 1;
  int DK = 0, K = 1;  // update kind and delay depth of the site's kernel
  size_t off, bytes;  // pool block
  // shared by the chains: descriptor, Weiss, initial fields, forced-flip
  // buffer, queue; per chain (chain 0's offsets, then + j * chain_stride):
  // fields, status, bins, state
  size_t o_desc, o_weiss, o_init, o_force, o_queue;
  size_t o_fields, o_bins, o_status, o_state, chain_stride;
  bool defined = false, has_state = false;
  bool busy = false;  // a serving request owns the site (guarded by the server mutex)
  hfqmc_problem prob{};
};

namespace {

enum ReqState { R_PENDING, R_READY, R_INFLIGHT, R_DONE };

struct Request {
  uint64_t ticket = 0;
  hfqmc_site* site = nullptr;
  hfqmc_problem prob{};
  // per chain: sweeps in all, sweeps done, sweeps of the step in flight
  std::vector<int64_t> total, done, q;
  int state = R_PENDING;
  bool first = true, given = false, keep = false, cancel = false;
  double weight = 0.0;
  hfqmc_status status = HFQMC_OK;
  std::vector<double> g[2], gerr[2], bins;
  std::vector<int8_t> fields;
  hfqmc_result res{};
};

struct Launch {
  int slot;
  int LT, RT, DK, K;  // kernel class
  int64_t max_props;  // largest q * L among the items (the launch's critical path)
  std::vector<Request*> items;
};

// Kernel class key of a site.
inline int64_t class_key(const hfqmc_site* s) {
  return ((int64_t)s->LT << 24) | ((int64_t)(s->RT & 0xff) << 16) | ((int64_t)s->DK << 8) | s->K;
}

struct Server {
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  bool started = false, stop = false, failed = false;
  std::string error;
  std::deque<Request*> pending;
  std::vector<Request*> ready;
  std::vector<Launch> inflight;  // the classes of the step in flight
  std::map<uint64_t, Request*> tickets;
  uint64_t next_ticket = 1;
  double used = 0.0;
  double capacity = 0.0;      // CU shares available to admitted requests
  double step_ms = 8.0;       // target duration of one step
  int64_t quantum = 0;        // > 0: fixed proposals per request per step instead
  int max_items = 2048;       // requests per class launch
  size_t max_pending = 1 << 16;
  hipStream_t streams[kSrvStreams] = {};
  hipEvent_t ev_begin[kSrvStreams] = {}, ev_end[kSrvStreams] = {};
  hipStream_t io = nullptr;
  size_t area_off = 0, area_bytes = 0, slot_bytes = 0;
  uint8_t* host_img[kSrvStreams] = {};
  int64_t submitted = 0, completed = 0, cancelled = 0, launches = 0, steps = 0;
  double step_ms_sum = 0.0, kernel_ms_sum = 0.0;  // wall time of steps, device time of class launches
  std::chrono::steady_clock::time_point step_t0;
};

}  // namespace

struct hfqmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hfqmc_precision prec = HFQMC_FP64;
  int n_cu = 0;
  std::mutex mu;
  // staged batch
  bool staged = false;
  uint8_t* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<hfqmc_problem> probs;  // as given (n_chains chains each)
  std::vector<int> item_owner, item_chain;  // work item -> (problem, chain)
  std::vector<int64_t> item_measure;        // measured sweeps of each item
  std::vector<Group> groups;
  Layout lo;
  hipStream_t aux[kAuxStreams] = {};
  hipStream_t cap = nullptr;  // capture stream for the graph
  hipEvent_t ev_fork = nullptr, ev_join[kAuxStreams] = {}, ev_start = nullptr, ev_end = nullptr;
  std::vector<hipEvent_t> ev;  // per group start/end
  hipGraphExec_t gexec = nullptr;
  int last_launches = 0;
  bool last_timed_groups = false;
  // tuning
  std::string tune_path;
  std::vector<TuneEntry> tune_all;  // every entry of the cache file
  std::map<int, TuneEntry> tune;    // this precision, by padded L
  // pool
  uint8_t* pool = nullptr;
  size_t pool_bytes = 0;
  std::vector<PoolBlock> free_list;
  std::vector<hfqmc_site*> sites;
  Server srv;
  // per-chain settings copied into every descriptor
  double drift_limit = 0.0;
  int64_t poison[2] = {0, 0};  // test hook: 1 + sweep, 0 = none
};

namespace {

// The context's per-chain settings into a descriptor (after fill_constants).
void apply_settings(ImpDesc& d, const hfqmc_ctx* c) {
  d.drift_limit = c->drift_limit;
  d.poison[0] = c->poison[0];
  d.poison[1] = c->poison[1];
}

hfqmc_status set_device(hfqmc_ctx* c) {
  HIP_TRY(hipSetDevice(c->device));
  return HFQMC_OK;
}

// The context's events (created with the context).
hfqmc_status ensure_base_events(hfqmc_ctx* c) {
  if (c->ev_start) return HFQMC_OK;
  for (int a = 0; a < kAuxStreams; ++a) HIP_TRY(hipEventCreateWithFlags(&c->ev_join[a], hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  HIP_TRY(hipEventCreate(&c->ev_end));
  HIP_TRY(hipEventCreate(&c->ev_start));
  return HFQMC_OK;
}

// The auxiliary streams the classes of a pass fork onto, and the capture
// stream, created at the first batch that uses them: every stream of a
// process takes one of its few hardware queues in turn, and streams created
// ahead of the serving engine's shift the engine's streams onto shared
// queues (measured: serving p50 134 ms without them, 901 ms with them).
hfqmc_status ensure_streams(hfqmc_ctx* c) {
  TRY(ensure_base_events(c));
  if (c->cap) return HFQMC_OK;
  for (int a = 0; a < kAuxStreams; ++a) HIP_TRY(hipStreamCreateWithFlags(&c->aux[a], hipStreamNonBlocking));
  HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
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

// Kernel shape for a problem: explicit delay, else the tuned entry of its
// class, else the default window-update kernel.
Plan plan_for(const hfqmc_ctx* c, const hfqmc_problem& p) {
  const int LT = padded_L(p.L);
  const int dk_delayed = c->prec == HFQMC_MIXED ? 2 : 1;
  const int dk_window = c->prec == HFQMC_MIXED ? kDkWindowMixed : kDkWindow;
  Plan pl;
  auto it = c->tune.find(LT);
  const bool tuned = it != c->tune.end();
  if (p.delay == 0 && tuned) {
    pl.k = it->second.k;
    pl.rt = it->second.rt;
    if (pl.k == 0)  // window updates; fp64 where no fp32-product variant exists
      pl.dk = LT <= kMaxRegisterL && find_kernel(window_LT(p.L), pl.rt, dk_window) ? dk_window : kDkWindow;
    else
      pl.dk = pl.rt == 0 ? 1 : (pl.k > 1 ? dk_delayed : 0);
  } else if (LT > kMaxRegisterL) {
    // G in device memory: fp64 window updates (delay 0), or fp64 delayed
    // updates of the given depth
    pl.rt = 0;
    if (p.delay == 0 && find_kernel(LT, 0, kDkWindow)) {
      pl.dk = kDkWindow;
      pl.k = 0;
    } else {
      pl.dk = 1;
      pl.k = p.delay >= 1 ? p.delay : kGlobalMaxDelay;
    }
  } else if (p.delay == 0 && (c->prec == HFQMC_MIXED || window_default(window_LT(p.L)))) {
    // mixed precision: the window kernel with fp32 flush products where one
    // is compiled for the class, else the fp64 one
    pl.k = 0;
    pl.rt = default_rt_window(window_LT(p.L), c->prec == HFQMC_MIXED);
    pl.dk = find_kernel(window_LT(p.L), pl.rt, dk_window) ? dk_window : kDkWindow;
  } else if (p.delay <= 1) {
    pl.rt = tuned && it->second.k == 1 ? it->second.rt : default_rt(LT, 0);
  } else {
    pl.k = p.delay;
    pl.dk = dk_delayed;
    pl.rt = tuned && it->second.k > 1 ? it->second.rt : default_rt(LT, pl.dk);
  }
  pl.LT = kernel_LT(p.L, pl.dk);
  return pl;
}

// Stage a batch: group by kernel class (padded L, shape), order items inside
// a class by descending work, upload descriptors and inputs.  `force`, when
// set, overrides the plan of every problem, or with force_LT of the problems
// of that padded L only, which then launch apart from the rest (autotuning:
// the class is timed beside the others).  `streams`: create the auxiliary
// streams the pass forks onto (not for the static entry point, which creates
// nothing and runs the classes in turn on the context stream).
hfqmc_status stage_impl(hfqmc_ctx* c, const hfqmc_problem* p0, int n0, void* d_ws, size_t ws_bytes,
                        const Plan* force, bool streams = true, int force_LT = 0) {
  for (int i = 0; i < n0; ++i) TRY(validate(p0[i], i));
  const Expanded ex = expand(p0, n0);  // from here on a work item is one chain
  const hfqmc_problem* p = ex.items.data();
  const int n = (int)ex.items.size();
  Layout lo = plan_layout(p, n);
  if (ws_bytes < lo.total) return fail(HFQMC_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, lo.total);
  TRY(set_device(c));
  TRY(streams ? ensure_streams(c) : ensure_base_events(c));
  if (c->gexec) {
    HIP_TRY(hipGraphExecDestroy(c->gexec));
    c->gexec = nullptr;
  }
  c->staged = false;

  std::vector<int> idx(n);
  std::vector<Plan> plan(n);
  std::vector<char> forced(n, 0);
  for (int i = 0; i < n; ++i) {
    idx[i] = i;
    forced[i] = force && (force_LT == 0 || padded_L(p[i].L) == force_LT);
    plan[i] = forced[i] ? *force : plan_for(c, p[i]);
    if (forced[i]) plan[i].LT = kernel_LT(p[i].L, plan[i].dk);
    if (plan[i].rt == 0 && plan[i].k > kGlobalMaxDelay)
      return fail(HFQMC_EINVAL, "problem %d: delay %d > %d for L=%d", ex.owner[i], plan[i].k, kGlobalMaxDelay, p[i].L);
    if (!find_kernel(plan[i].LT, plan[i].rt, plan[i].dk))
      return fail(HFQMC_EINVAL, "problem %d: no %s kernel for L=%d", ex.owner[i],
                  plan[i].dk ? "delayed-update" : "sweep", p[i].L);
  }
  // expected work: sweeps x L proposals, a fraction exp(-0.76 lambda^2) of
  // them accepted (fits the measured acceptance of the chain workloads at
  // both ends of U in [4, 12]), each accept about max(L, 64) units.  The
  // heaviest items start first; when all items are resident at once this
  // also places the heaviest beside the lightest (measured: 97 -> 85 ms on
  // the 512 x L = 64 batch with U in [4, 12])
  auto cost = [&](int i) {
    const double lam = coupling(p[i].beta / p[i].L, p[i].U);
    return (double)(p[i].n_warmup + p[i].n_measure) * p[i].L * std::max(p[i].L, 64) * std::exp(-0.76 * lam * lam);
  };
  // the class an autotuning run times keeps launches of its own
  auto key = [&](int i) { return std::make_tuple(-plan[i].LT, plan[i].dk, plan[i].rt, force_LT && forced[i]); };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (key(a) != key(b)) return key(a) < key(b);
    return cost(a) > cost(b);
  });
  std::vector<Group> groups;
  for (int k = 0; k < n;) {
    int e = k;
    while (e < n && key(idx[e]) == key(idx[k])) ++e;
    const Plan& pl = plan[idx[k]];
    const int LT = pl.LT;
    const KernelInfo* ki = find_kernel(LT, pl.rt, pl.dk);
    int bpc = 0;
    HIP_TRY(kernel_occupancy(ki, &bpc));
    if (bpc < 1) return fail(HFQMC_EDEVICE, "kernel for L=%d does not fit on a CU", LT);
    groups.push_back({ki, LT, pl.rt, pl.dk, k, e - k, std::min(e - k, bpc * c->n_cu)});
    groups.back().tuned = force_LT && forced[idx[k]];
    k = e;
  }
  if (groups.size() > 64) return fail(HFQMC_EINVAL, "too many kernel classes");
  // Streams of the classes: longest expected class first, each onto the
  // stream with the least expected work so far, so that a short class does
  // not queue behind the longest one when there are more classes than
  // streams (measured on the uneven batch: the 32-slice class after the
  // 128-slice one made the pass 232 ms instead of 206).  Expected duration:
  // the heaviest item, or the class's work spread over its resident items.
  {
    const int G = (int)groups.size();
    const int ns = streams ? std::min(G, 1 + kAuxStreams) : 1;
    std::vector<double> est(G);
    for (int g = 0; g < G; ++g) {
      double sum = 0.0;
      for (int i = groups[g].first; i < groups[g].first + groups[g].count; ++i) sum += cost(idx[i]);
      est[g] = std::max(cost(idx[groups[g].first]), sum / groups[g].grid);
    }
    std::vector<int> by(G);
    for (int g = 0; g < G; ++g) by[g] = g;
    std::stable_sort(by.begin(), by.end(), [&](int a, int b) { return est[a] > est[b]; });
    std::vector<double> load(ns, 0.0);
    for (int g : by) {
      const int st = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      groups[g].stream = st;
      load[st] += est[g];
    }
  }

  // host image of the input region [descs, status)
  std::vector<uint8_t> img(lo.status, 0);
  ImpDesc* descs = reinterpret_cast<ImpDesc*>(img.data() + lo.descs);
  int32_t* order = reinterpret_cast<int32_t*>(img.data() + lo.order);
  for (int i = 0; i < n; ++i) {
    ImpDesc d{};
    fill_constants(d, p[i]);
    apply_settings(d, c);
    d.LT = plan[i].LT;
    d.op = OP_SWEEPS;
    d.delay = plan[i].k;
    d.flags = F_ZERO_ACC | (p[i].init_fields ? F_FIELDS_GIVEN : 0) | F_SAVE;
    d.off_weiss = (int64_t)lo.w_off[i];
    d.off_init = (int64_t)lo.i_off[i];
    d.off_fields = (int64_t)lo.f_off[i];
    d.off_bins = (int64_t)lo.b_off[i];
    d.off_status = (int64_t)(lo.status + sizeof(ImpStatus) * i);
    d.off_state = (int64_t)lo.s_off[i];
    d.off_force = 0;
    d.chain = ex.chain[i];
    descs[i] = d;
    std::memcpy(img.data() + lo.w_off[i], p[i].weiss[0], sizeof(double) * p[i].L);
    std::memcpy(img.data() + lo.w_off[i] + sizeof(double) * p[i].L, p[i].weiss[1], sizeof(double) * p[i].L);
    if (p[i].init_fields) std::memcpy(img.data() + lo.i_off[i], p[i].init_fields, p[i].L);
  }
  for (int i = 0; i < n; ++i) order[i] = idx[i];
  c->ws = reinterpret_cast<uint8_t*>(d_ws);
  c->ws_bytes = ws_bytes;
  HIP_TRY(hipMemcpyAsync(c->ws, img.data(), img.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->probs.assign(p0, p0 + n0);
  for (auto& q : c->probs) q.weiss[0] = q.weiss[1] = nullptr, q.init_fields = nullptr;
  c->item_owner = ex.owner;
  c->item_chain = ex.chain;
  c->item_measure.resize(n);
  for (int i = 0; i < n; ++i) c->item_measure[i] = p[i].n_measure;
  c->groups = groups;
  c->lo = lo;
  c->staged = true;
  return HFQMC_OK;
}

// Enqueue one whole pass on `main`: reset the work queues, then every class
// kernel, classes spread over the auxiliary streams so that they run
// concurrently (fork/join through events; valid under stream capture).  No
// memset and no host copy: the pass can be captured into a graph.
hfqmc_status enqueue_pass(hfqmc_ctx* c, hipStream_t main, bool timing) {
  const int G = (int)c->groups.size();
  // without the auxiliary streams (the static entry point) the classes run
  // one after another on `main`
  const int ns = c->cap ? std::min(G, 1 + kAuxStreams) : 1;
  if (timing) TRY(ensure_events(c, 2 * (size_t)G));
  HIP_TRY(launch_zero(c->ws + c->lo.queues, sizeof(int32_t) * 64, main));
  if (ns > 1) {
    HIP_TRY(hipEventRecord(c->ev_fork, main));
    for (int a = 0; a < ns - 1; ++a) HIP_TRY(hipStreamWaitEvent(c->aux[a], c->ev_fork, 0));
  }
  const ImpDesc* descs = reinterpret_cast<const ImpDesc*>(c->ws + c->lo.descs);
  const int32_t* order = reinterpret_cast<const int32_t*>(c->ws + c->lo.order);
  int* queues = reinterpret_cast<int*>(c->ws + c->lo.queues);
  for (int gi = 0; gi < G; ++gi) {
    const Group& gr = c->groups[gi];
    const int si = gr.stream % ns;
    hipStream_t st = si == 0 ? main : c->aux[si - 1];
    if (timing) HIP_TRY(hipEventRecord(c->ev[2 * gi], st));
    HIP_TRY(launch_sweep(gr.k, gr.grid, st, descs, order + gr.first, gr.count, queues + gi, c->ws));
    if (timing) HIP_TRY(hipEventRecord(c->ev[2 * gi + 1], st));
  }
  if (ns > 1) {
    for (int a = 0; a < ns - 1; ++a) {
      HIP_TRY(hipEventRecord(c->ev_join[a], c->aux[a]));
      HIP_TRY(hipStreamWaitEvent(main, c->ev_join[a], 0));
    }
  }
  return HFQMC_OK;
}

// Per-pass device time (ms) from the start/end events on the context stream.
hfqmc_status pass_ms(hfqmc_ctx* c, double* ms) {
  HIP_TRY(hipEventSynchronize(c->ev_end));
  float t = 0.f;
  HIP_TRY(hipEventElapsedTime(&t, c->ev_start, c->ev_end));
  *ms = t;
  return HFQMC_OK;
}

// ---- serving helpers (the server mutex is held by the caller) ----

size_t site_layout(hfqmc_site* s) {
  size_t off = 0;
  s->o_desc = off;
  off = align_up(off + sizeof(ImpDesc), 256);
  s->o_weiss = off;
  off = align_up(off + sizeof(double) * 2 * s->L, 256);
  s->o_init = off;
  off = align_up(off + s->L, 256);
  s->o_force = off;
  off = align_up(off + 1024 * (sizeof(int32_t) + sizeof(double)), 256);
  s->o_queue = off;  // queue counter + order entry
  off = align_up(off + 256, 256);
  const size_t chain0 = off;
  s->o_fields = off;
  off = align_up(off + s->L, 256);
  s->o_status = off;
  off = align_up(off + sizeof(ImpStatus), 256);
  s->o_bins = off;
  off = align_up(off + sizeof(double) * (size_t)s->n_bins * n_values(s->L), 256);
  s->o_state = off;
  off = align_up(off + state_bytes(s->L), 256);
  s->chain_stride = off - chain0;
  return chain0 + s->chain_stride * s->n_chains;
}

void site_offsets(const hfqmc_site* s, ImpDesc& d, int chain = 0) {
  const size_t cj = s->off + s->chain_stride * chain;
  d.off_weiss = (int64_t)(s->off + s->o_weiss);
  d.off_init = (int64_t)(s->off + s->o_init);
  d.off_fields = (int64_t)(cj + s->o_fields);
  d.off_bins = (int64_t)(cj + s->o_bins);
  d.off_status = (int64_t)(cj + s->o_status);
  d.off_state = (int64_t)(cj + s->o_state);
  d.off_force = (int64_t)(s->off + s->o_force);
  d.LT = s->LT;
  d.delay = s->K;
  d.chain = chain;
}

// Launch one work item on chain `chain` of a site (blocking, context stream).
hfqmc_status site_launch(hfqmc_ctx* c, hfqmc_site* s, ImpDesc d, int chain = 0) {
  uint8_t* base = c->pool + s->off;
  site_offsets(s, d, chain);
  const KernelInfo* k = find_kernel(s->LT, s->RT, s->DK);
  if (!k) return fail(HFQMC_EINVAL, "no kernel for LT=%d RT=%d", s->LT, s->RT);
  struct {
    int32_t queue, order;
  } qo = {0, 0};
  HIP_TRY(hipMemcpyAsync(base + s->o_desc, &d, sizeof d, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(base + s->o_queue, &qo, sizeof qo, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(launch_sweep(k, 1, c->stream, reinterpret_cast<const ImpDesc*>(base + s->o_desc),
                       reinterpret_cast<const int32_t*>(base + s->o_queue + 4), 1,
                       reinterpret_cast<int*>(base + s->o_queue), c->pool));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return HFQMC_OK;
}

// Blocks per CU of a site's kernel (its admission weight is 1 / that).
int site_bpc(const hfqmc_site* s) {
  const KernelInfo* k = find_kernel(s->LT, s->RT, s->DK);
  int bpc = 0;
  if (!k || kernel_occupancy(k, &bpc) != hipSuccess || bpc < 1) return 1;
  return bpc;
}

// Copy a finished request's bins, status and fields back, pool its chains
// and finalise them.
hfqmc_status srv_finish(hfqmc_ctx* c, Request* r) {
  Server& S = c->srv;
  hfqmc_site* s = r->site;
  const int L = s->L, NV = n_values(L), nb = s->n_bins, nc = s->n_chains;
  std::vector<double> part((size_t)nc * nb * NV), sums((size_t)nb * NV, 0.0);
  std::vector<ImpStatus> parts(nc);
  std::vector<int64_t> cnt(nb, 0);
  ImpStatus st{};
  r->fields.resize(L);
  uint8_t* base = c->pool + s->off;
  for (int j = 0; j < nc; ++j) {
    const size_t cj = s->chain_stride * j;
    HIP_TRY(hipMemcpyAsync(&part[(size_t)j * nb * NV], base + cj + s->o_bins, sizeof(double) * nb * NV,
                           hipMemcpyDeviceToHost, S.io));
    HIP_TRY(hipMemcpyAsync(&parts[j], base + cj + s->o_status, sizeof(ImpStatus), hipMemcpyDeviceToHost, S.io));
  }
  HIP_TRY(hipMemcpyAsync(r->fields.data(), base + s->o_fields, L, hipMemcpyDeviceToHost, S.io));
  HIP_TRY(hipStreamSynchronize(S.io));
  for (int j = 0; j < nc; ++j) {
    pool_chain(NV, nb, &part[(size_t)j * nb * NV], parts[j], sums.data(), st);
    add_bin_counts(chain_measure(r->prob, j), nb, cnt.data());
  }
  for (int k = 0; k < 2; ++k) {
    r->g[k].assign(L + 1, 0.0);
    r->gerr[k].assign(L + 1, 0.0);
    r->res.g[k] = r->g[k].data();
    r->res.g_err[k] = r->gerr[k].data();
  }
  r->bins.assign(sums.size(), 0.0);
  r->res.bins = r->bins.data();
  r->res.final_fields = nullptr;
  finalise(L, nb, sums.data(), cnt.data(), st, r->fields.data(), r->res);
  r->status = (hfqmc_status)r->res.status;
  return HFQMC_OK;
}

// Time per proposal of one chain of a kernel class, as measured on MI355X
// with one or two impurities per CU (512-impurity classes of the chain
// workload, 2200 sweeps): 0.4 us at 32 slices, 0.55 us at 48-64 (rank-one
// kernels), 0.85 us at 80, 0.5 - 0.6 us at 96-128 (window kernels), 1.35 us
// at L = 160 on the device-memory kernel.  Used to give every class about
// `step_ms` of work per step.
double model_us_per_proposal(const hfqmc_site* s) {
  if (s->RT == 0) return 1.35 * s->L / 160.0;
  if (s->LT <= 32) return 0.4;
  if (s->LT <= 64) return 0.55;
  if (s->LT <= 80) return 0.85;
  return 0.6;
}

// One pass of the engine.  Work advances in lockstep steps: a step launches
// every admitted request once, each kernel class on its own stream, with a
// per-class sweep count sized from that class's measured time per proposal
// so that every class kernel takes about `step_ms`.  When all kernels of the
// step have finished, its requests retire or become ready again, queued
// requests are admitted, and the next step starts.  Returns true while a
// step is in flight.
bool srv_step(hfqmc_ctx* c) {
  Server& S = c->srv;
  auto device_fail = [&](const char* what, hipError_t e) {
    S.failed = true;
    S.error = std::string(what) + ": " + hipGetErrorString(e);
  };
  // 1. retire the step once every class kernel of it has finished
  if (!S.inflight.empty()) {
    for (const Launch& L : S.inflight) {
      const hipError_t q = hipEventQuery(S.ev_end[L.slot]);
      if (q == hipErrorNotReady) return true;
      if (q != hipSuccess) device_fail("hipEventQuery", q);
    }
    S.step_ms_sum += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - S.step_t0).count();
    for (Launch& L : S.inflight) {
      float ms = 0.f;
      if (!S.failed && hipEventElapsedTime(&ms, S.ev_begin[L.slot], S.ev_end[L.slot]) == hipSuccess)
        S.kernel_ms_sum += ms;
      for (Request* r : L.items) {
        bool finished = true;
        for (size_t j = 0; j < r->q.size(); ++j) {
          r->done[j] += r->q[j];
          r->q[j] = 0;
          finished = finished && r->done[j] >= r->total[j];
        }
        r->first = false;
        if (r->cancel) {
          S.used -= r->weight;
          r->site->busy = false;
          r->site->has_state = true;
          S.tickets.erase(r->ticket);
          ++S.cancelled;
          delete r;
        } else if (S.failed || finished) {
          S.used -= r->weight;
          if (S.failed) {
            r->status = HFQMC_EDEVICE;
          } else if (srv_finish(c, r) != HFQMC_OK) {
            S.failed = true;
            S.error = t_err;
            r->status = HFQMC_EDEVICE;
          }
          r->state = R_DONE;
          r->site->busy = false;
          r->site->has_state = true;
          ++S.completed;
        } else {
          r->state = R_READY;
          S.ready.push_back(r);
        }
      }
    }
    S.inflight.clear();
  }
  if (S.failed) {
    for (Request* r : S.ready) {
      S.used -= r->weight;
      r->status = HFQMC_EDEVICE;
      r->state = R_DONE;
      r->site->busy = false;
    }
    S.ready.clear();
    return false;
  }
  if (S.stop) return false;
  // 2. admit in arrival order; a request that does not fit lets smaller
  // later ones pass
  for (auto it = S.pending.begin(); it != S.pending.end();) {
    Request* r = *it;
    if (S.used + r->weight <= S.capacity + 1e-9 || S.used <= 1e-9) {
      S.used += r->weight;
      r->state = R_READY;
      S.ready.push_back(r);
      it = S.pending.erase(it);
    } else {
      ++it;
    }
  }
  if (S.ready.empty()) return false;
  // 3. the next step: one launch per kernel class
  std::map<int64_t, std::vector<Request*>> classes;
  for (Request* r : S.ready) classes[class_key(r->site)].push_back(r);
  std::vector<Request*> left;
  int slot = 0;
  for (auto& kv : classes) {
    std::vector<Request*>& v = kv.second;
    if (slot == kSrvStreams) {  // more classes than streams: the rest waits a step
      left.insert(left.end(), v.begin(), v.end());
      continue;
    }
    // one work item per unfinished chain; a request's chains go together
    size_t take = 0;
    int n = 0;
    for (; take < v.size(); ++take) {
      int u = 0;
      for (size_t j = 0; j < v[take]->total.size(); ++j) u += v[take]->done[j] < v[take]->total[j];
      if (n + u > S.max_items && take > 0) break;
      n += u;
    }
    if (take < v.size()) {
      left.insert(left.end(), v.begin() + take, v.end());
      v.resize(take);
    }
    const hfqmc_site* head = v.front()->site;
    Launch L{slot, head->LT, head->RT, head->DK, head->K, 0, v};
    const double us = model_us_per_proposal(head);
    uint8_t* img = S.host_img[slot];
    ImpDesc* descs = reinterpret_cast<ImpDesc*>(img);
    int32_t* order = reinterpret_cast<int32_t*>(img + align_up(sizeof(ImpDesc) * S.max_items, 256));
    int32_t* queue = order + S.max_items;
    const int64_t props = S.quantum > 0 ? S.quantum : (int64_t)(1e3 * S.step_ms / us);
    int i = 0;
    for (Request* r : v) {
      const int64_t q = std::max<int64_t>(1, props / r->site->L);
      for (int j = 0; j < (int)r->total.size(); ++j) {
        r->q[j] = std::min(q, r->total[j] - r->done[j]);
        if (r->q[j] == 0) continue;
        ImpDesc d{};
        fill_constants(d, r->prob);
        apply_settings(d, c);
        site_offsets(r->site, d, j);
        d.op = OP_SWEEPS;
        d.n_measure = chain_measure(r->prob, j);
        L.max_props = std::max(L.max_props, r->q[j] * r->site->L);
        d.sweep_begin = r->done[j];
        d.sweep_end = r->done[j] + r->q[j];
        if (r->first)
          d.flags = F_ZERO_ACC | F_SAVE | F_SAVE_G | (r->given ? F_FIELDS_GIVEN : (r->keep ? F_KEEP_FIELDS : 0));
        else
          d.flags = F_RESUME | F_SAVE | F_SAVE_G;
        descs[i] = d;
        order[i] = i;
        ++i;
      }
      r->state = R_INFLIGHT;
    }
    *queue = 0;
    uint8_t* dev = c->pool + S.area_off + (size_t)slot * S.slot_bytes;
    const size_t bytes = reinterpret_cast<uint8_t*>(queue + 1) - img;
    const KernelInfo* k = find_kernel(L.LT, L.RT, L.DK);
    int bpc = 1;
    hipError_t e = kernel_occupancy(k, &bpc);
    if (e == hipSuccess) e = hipMemcpyAsync(dev, img, bytes, hipMemcpyHostToDevice, S.streams[slot]);
    if (e == hipSuccess) e = hipEventRecord(S.ev_begin[slot], S.streams[slot]);
    if (e == hipSuccess)
      e = launch_sweep(k, std::min(n, std::max(1, bpc) * c->n_cu), S.streams[slot], reinterpret_cast<const ImpDesc*>(dev),
                       reinterpret_cast<const int32_t*>(dev + (reinterpret_cast<uint8_t*>(order) - img)), n,
                       reinterpret_cast<int*>(dev + (reinterpret_cast<uint8_t*>(queue) - img)), c->pool);
    if (e == hipSuccess) e = hipEventRecord(S.ev_end[slot], S.streams[slot]);
    if (e != hipSuccess) device_fail("serving launch", e);
    S.inflight.push_back(std::move(L));
    ++S.launches;
    ++slot;
  }
  S.ready.swap(left);
  ++S.steps;
  S.step_t0 = std::chrono::steady_clock::now();
  return true;
}

void srv_main(hfqmc_ctx* c) {
  Server& S = c->srv;
  (void)hipSetDevice(c->device);
  std::unique_lock<std::mutex> lk(S.mu);
  for (;;) {
    const bool busy = srv_step(c);
    if (S.stop && !busy) break;
    if (busy)
      S.cv.wait_for(lk, std::chrono::microseconds(50));
    else
      S.cv.wait(lk, [&] { return S.stop || !S.pending.empty() || !S.ready.empty(); });
  }
}

// Streams, pinned launch images and the device launch area (from the pool);
// the context mutex is held.
hfqmc_status srv_start(hfqmc_ctx* c) {
  Server& S = c->srv;
  if (S.started) return HFQMC_OK;
  TRY(set_device(c));
  S.slot_bytes = align_up(align_up(sizeof(ImpDesc) * S.max_items, 256) + sizeof(int32_t) * (S.max_items + 1), 256);
  S.area_bytes = S.slot_bytes * kSrvStreams;
  TRY(pool_alloc(c, S.area_bytes, &S.area_off));
  for (int k = 0; k < kSrvStreams; ++k) {
    HIP_TRY(hipStreamCreateWithFlags(&S.streams[k], hipStreamNonBlocking));
    HIP_TRY(hipEventCreate(&S.ev_begin[k]));
    HIP_TRY(hipEventCreate(&S.ev_end[k]));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&S.host_img[k]), S.slot_bytes, hipHostMallocDefault));
  }
  HIP_TRY(hipStreamCreateWithFlags(&S.io, hipStreamNonBlocking));
  if (S.capacity <= 0.0) S.capacity = (double)c->n_cu;
  S.stop = false;
  S.th = std::thread(srv_main, c);
  S.started = true;
  return HFQMC_OK;
}

void srv_shutdown(hfqmc_ctx* c) {
  Server& S = c->srv;
  if (!S.started) return;
  {
    std::lock_guard<std::mutex> g(S.mu);
    S.stop = true;  // launches in flight drain, nothing new starts
  }
  S.cv.notify_all();
  S.th.join();
  for (auto& kv : S.tickets) delete kv.second;  // every live request holds a ticket
  S.tickets.clear();
  S.pending.clear();
  S.ready.clear();
  for (int k = 0; k < kSrvStreams; ++k) {
    (void)hipStreamDestroy(S.streams[k]);
    (void)hipEventDestroy(S.ev_begin[k]);
    (void)hipEventDestroy(S.ev_end[k]);
    (void)hipHostFree(S.host_img[k]);
  }
  (void)hipStreamDestroy(S.io);
  S.started = false;
}

bool site_known(hfqmc_ctx* c, hfqmc_site* s) { return std::find(c->sites.begin(), c->sites.end(), s) != c->sites.end(); }

bool site_busy(hfqmc_ctx* c, hfqmc_site* s) {
  std::lock_guard<std::mutex> g(c->srv.mu);
  return s->busy;
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
  c->drift_limit = precision == HFQMC_MIXED ? kMixedDriftLimit : 0.0;
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
  // set-up for hfqmc_solve_static, with the device current: the static
  // array's device address, and the streams and events every pass uses, so
  // that call creates and allocates nothing
  if (hfqmc_status st = scratch_setup(device)) {
    delete c;
    return st;
  }
  if (hfqmc_status st = ensure_base_events(c)) {
    delete c;
    return st;
  }
  if (tune_cache) {
    c->tune_path = tune_cache;
    c->tune_all = read_tune_cache(c->tune_path);
    for (const auto& t : c->tune_all) {
      if (t.prec != prec_name(precision)) continue;
      if (t.k == 0) {  // window updates
        const int dk = precision == HFQMC_MIXED ? kDkWindowMixed : kDkWindow;
        if (t.LT <= kMaxRegisterL ? find_kernel(window_LT(t.LT), t.rt, dk) != nullptr
                                  : (t.rt == 0 && find_kernel(t.LT, 0, kDkWindow) != nullptr))
          c->tune[t.LT] = t;
        continue;
      }
      const int dk = t.rt == 0 ? 1 : (t.k > 1 ? (precision == HFQMC_MIXED ? 2 : 1) : 0);
      const int kmax = t.rt == 0 ? kGlobalMaxDelay : kMaxDelay;
      if (t.k >= 1 && t.k <= kmax && find_kernel(t.LT, t.rt, dk)) c->tune[t.LT] = t;
    }
  }
  *out = c;
  return HFQMC_OK;
}

void hfqmc_destroy(hfqmc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  srv_shutdown(c);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  for (auto e : c->ev) (void)hipEventDestroy(e);
  if (c->cap) {
    for (int a = 0; a < kAuxStreams; ++a) (void)hipStreamDestroy(c->aux[a]);
    (void)hipStreamDestroy(c->cap);
  }
  if (c->ev_start) {
    for (int a = 0; a < kAuxStreams; ++a) (void)hipEventDestroy(c->ev_join[a]);
    (void)hipEventDestroy(c->ev_fork);
    (void)hipEventDestroy(c->ev_start);
    (void)hipEventDestroy(c->ev_end);
  }
  for (auto s : c->sites) delete s;
  delete c;
}

const char* hfqmc_last_error(const hfqmc_ctx*) { return t_err.c_str(); }

hfqmc_status hfqmc_workspace_size(hfqmc_ctx* c, const hfqmc_problem* p, int32_t n, size_t* bytes) {
  if (!c || !bytes || n < 0 || (n > 0 && !p)) return fail(HFQMC_EINVAL, "hfqmc_workspace_size: bad arguments");
  for (int i = 0; i < n; ++i) TRY(validate(p[i], i));
  const Expanded ex = expand(p, n);
  *bytes = plan_layout(ex.items.data(), (int)ex.items.size()).total;
  return HFQMC_OK;
}

hfqmc_status hfqmc_stage(hfqmc_ctx* c, const hfqmc_problem* p, int32_t n, void* d_ws, size_t ws_bytes) {
  if (!c || n < 1 || !p || !d_ws) return fail(HFQMC_EINVAL, "hfqmc_stage: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  return stage_impl(c, p, n, d_ws, ws_bytes, nullptr);
}

hfqmc_status hfqmc_run(hfqmc_ctx* c) {
  if (!c || !c->staged) return fail(HFQMC_EINVAL, "hfqmc_run: nothing staged");
  std::lock_guard<std::mutex> g(c->mu);
  TRY(set_device(c));
  HIP_TRY(hipEventRecord(c->ev_start, c->stream));
  TRY(enqueue_pass(c, c->stream, true));
  HIP_TRY(hipEventRecord(c->ev_end, c->stream));
  c->last_launches = (int)c->groups.size();
  c->last_timed_groups = true;
  return HFQMC_OK;
}

hfqmc_status hfqmc_set_drift_limit(hfqmc_ctx* c, double limit) {
  if (!c || !(limit >= 0.0) || !std::isfinite(limit)) return fail(HFQMC_EINVAL, "hfqmc_set_drift_limit: need limit >= 0");
  std::lock_guard<std::mutex> g(c->mu);
  c->drift_limit = limit;
  return HFQMC_OK;
}

hfqmc_status hfqmc_debug_poison(hfqmc_ctx* c, int64_t sweep_a, int64_t sweep_b) {
  if (!c || sweep_a < -1 || sweep_b < -1) return fail(HFQMC_EINVAL, "hfqmc_debug_poison: sweeps must be >= -1");
  std::lock_guard<std::mutex> g(c->mu);
  c->poison[0] = sweep_a + 1;
  c->poison[1] = sweep_b + 1;
  return HFQMC_OK;
}

hfqmc_status hfqmc_solve_static(hfqmc_ctx* c, const hfqmc_problem* p, int32_t n, hfqmc_result* out) {
  if (c && n == 0) return HFQMC_OK;  // an empty batch: nothing to run
  if (!c || !p || n < 1 || !out) return fail(HFQMC_EINVAL, "hfqmc_solve_static: bad arguments");
  size_t need = 0;
  TRY(hfqmc_workspace_size(c, p, n, &need));
  if (need > HFQMC_STATIC_BYTES)
    return fail(HFQMC_EINVAL, "hfqmc_solve_static: the batch needs %zu bytes of workspace, the static array holds %zu",
                need, (size_t)HFQMC_STATIC_BYTES);
  void* ws = scratch_ptr(c->device);
  if (!ws) return fail(HFQMC_EDEVICE, "hfqmc_solve_static: no static array on device %d", c->device);
  {
    std::lock_guard<std::mutex> g(c->mu);
    TRY(stage_impl(c, p, n, ws, HFQMC_STATIC_BYTES, nullptr, false));
    TRY(set_device(c));
    // the whole pass, timed only by the start/end events created with the context
    HIP_TRY(hipEventRecord(c->ev_start, c->stream));
    TRY(enqueue_pass(c, c->stream, false));
    HIP_TRY(hipEventRecord(c->ev_end, c->stream));
    c->last_launches = (int)c->groups.size();
    c->last_timed_groups = false;
  }
  return hfqmc_collect(c, out);
}

hfqmc_status hfqmc_run_graph(hfqmc_ctx* c) {
  if (!c || !c->staged) return fail(HFQMC_EINVAL, "hfqmc_run_graph: nothing staged");
  std::lock_guard<std::mutex> g(c->mu);
  TRY(set_device(c));
  TRY(ensure_streams(c));
  if (!c->gexec) {
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    const hfqmc_status st = enqueue_pass(c, c->cap, false);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap, &graph);
    if (st != HFQMC_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (st != HFQMC_OK) return st;
      HIP_TRY(e);
    }
    const hipError_t ei = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIP_TRY(ei);
  }
  HIP_TRY(hipEventRecord(c->ev_start, c->stream));
  HIP_TRY(hipGraphLaunch(c->gexec, c->stream));
  HIP_TRY(hipEventRecord(c->ev_end, c->stream));
  c->last_launches = (int)c->groups.size();
  c->last_timed_groups = false;
  return HFQMC_OK;
}

hfqmc_status hfqmc_last_run_ms(hfqmc_ctx* c, double* ms, int32_t* n_launches) {
  if (!c || !ms) return fail(HFQMC_EINVAL, "hfqmc_last_run_ms: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (c->last_launches == 0) return fail(HFQMC_EINVAL, "no run recorded");
  TRY(pass_ms(c, ms));
  if (n_launches) *n_launches = c->last_launches;
  return HFQMC_OK;
}

hfqmc_status hfqmc_last_launch_ms(hfqmc_ctx* c, int32_t i, double* ms, int32_t* L_padded, int32_t* n_items) {
  if (!c || !ms) return fail(HFQMC_EINVAL, "hfqmc_last_launch_ms: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (c->last_launches == 0 || !c->last_timed_groups)
    return fail(HFQMC_EINVAL, "no eagerly launched run recorded (graph replays time the whole pass only)");
  if (i < 0 || i >= c->last_launches) return fail(HFQMC_EINVAL, "launch %d outside [0,%d)", i, c->last_launches);
  HIP_TRY(hipEventSynchronize(c->ev[2 * i + 1]));
  float t = 0.f;
  HIP_TRY(hipEventElapsedTime(&t, c->ev[2 * i], c->ev[2 * i + 1]));
  *ms = t;
  if (L_padded) *L_padded = c->groups[i].LT;
  if (n_items) *n_items = c->groups[i].count;
  return HFQMC_OK;
}

hfqmc_status hfqmc_collect(hfqmc_ctx* c, hfqmc_result* out) {
  if (!c || !c->staged || !out) return fail(HFQMC_EINVAL, "hfqmc_collect: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  TRY(set_device(c));
  const size_t lo_off = c->lo.fields, hi_off = c->lo.state;
  std::vector<uint8_t> host(hi_off - lo_off);
  HIP_TRY(hipMemcpyAsync(host.data(), c->ws + lo_off, hi_off - lo_off, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  hfqmc_status worst = HFQMC_OK;
  // items of one problem are consecutive, chain 0 first
  const size_t n_items = c->item_owner.size();
  for (size_t k = 0; k < n_items;) {
    const int i = c->item_owner[k];
    const hfqmc_problem& p = c->probs[i];
    const int NV = n_values(p.L), nb = p.n_bins;
    std::vector<double> sums((size_t)nb * NV, 0.0);
    std::vector<int64_t> cnt(nb, 0);
    ImpStatus st{};
    const int8_t* fields = reinterpret_cast<const int8_t*>(host.data() + (c->lo.f_off[k] - lo_off));
    for (; k < n_items && c->item_owner[k] == i; ++k) {
      pool_chain(NV, nb, reinterpret_cast<const double*>(host.data() + (c->lo.b_off[k] - lo_off)),
                 *reinterpret_cast<const ImpStatus*>(host.data() + (c->lo.status - lo_off) + sizeof(ImpStatus) * k),
                 sums.data(), st);
      add_bin_counts(c->item_measure[k], nb, cnt.data());
    }
    finalise(p.L, nb, sums.data(), cnt.data(), st, fields, out[i]);
    if (out[i].status != HFQMC_OK) worst = (hfqmc_status)out[i].status;
  }
  if (worst != HFQMC_OK) return fail(worst, "non-finite ratio or Green function in at least one impurity");
  return HFQMC_OK;
}

hfqmc_status hfqmc_solve(hfqmc_ctx* c, const hfqmc_problem* p, int32_t n, void* d_ws, size_t ws_bytes,
                         hfqmc_result* out) {
  if (c && n == 0) return HFQMC_OK;  // an empty batch: nothing to run
  if (!out) return fail(HFQMC_EINVAL, "hfqmc_solve: out is NULL");
  TRY(hfqmc_stage(c, p, n, d_ws, ws_bytes));
  TRY(hfqmc_run(c));
  return hfqmc_collect(c, out);
}

// ---------------------------------------------------------------- tuning

hfqmc_status hfqmc_tune(hfqmc_ctx* c, const hfqmc_problem* p, int32_t n, void* d_ws, size_t ws_bytes,
                        int32_t sweeps) {
  if (!c || !p || n < 1 || !d_ws || sweeps < 4) return fail(HFQMC_EINVAL, "hfqmc_tune: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  for (int i = 0; i < n; ++i) TRY(validate(p[i], i));
  std::vector<int> classes;
  for (int i = 0; i < n; ++i) classes.push_back(padded_L(p[i].L));
  std::sort(classes.begin(), classes.end());
  classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
  const int dk_delayed = c->prec == HFQMC_MIXED ? 2 : 1;
  // the whole batch with shortened chains (same Weiss, U, beta, seeds), at
  // two lengths: a class's rate is taken from the difference, so the
  // per-launch costs that a full-length run amortises (the first Dyson
  // solve, the launch itself) do not decide between shapes.  Every class
  // runs in each timing run, as in a pass, so a shape is timed beside the
  // classes it will share the CUs with (alone, with one impurity per CU, a
  // shape with more waves can win and then lose beside the others)
  std::vector<hfqmc_problem> sample, sample2;
  for (int i = 0; i < n; ++i) {
    hfqmc_problem q = p[i];
    q.n_warmup = sweeps / 2;
    q.n_measure = (int64_t)(sweeps - sweeps / 2) * chains_of(q);
    q.n_bins = std::min(q.n_bins, 2);
    sample.push_back(q);
    q.n_warmup = sweeps;
    q.n_measure = (int64_t)sweeps * chains_of(q);
    sample2.push_back(q);
  }
  for (int LT : classes) {
    int64_t props = 0;  // the difference of the two lengths
    int first = -1;
    for (int i = 0; i < n; ++i)
      if (padded_L(p[i].L) == LT) {
        props += (int64_t)sweeps * p[i].L * chains_of(p[i]);
        if (first < 0) first = i;
      }
    std::vector<Plan> cands;
    int rts[16];
    if (LT <= kMaxRegisterL) {  // window updates (k = 0 in the cache)
      const int dk_window = c->prec == HFQMC_MIXED ? kDkWindowMixed : kDkWindow;
      const int nw = std::min(16, kernel_variants(window_LT(LT), dk_window, rts, 16));
      for (int v = 0; v < nw; ++v) cands.push_back({rts[v], dk_window, 0});
    }
    int nv = std::min(16, kernel_variants(LT, 0, rts, 16));
    for (int v = 0; v < nv; ++v) cands.push_back({rts[v], 0, 1});
    nv = std::min(16, kernel_variants(LT, dk_delayed, rts, 16));
    for (int v = 0; v < nv; ++v)
      for (int k : {4, 8, 16, 32})
        if (rts[v] != 0) cands.push_back({rts[v], dk_delayed, k});
    if (find_kernel(LT, 0, kDkWindow))  // device-memory window updates (fp64 in either precision)
      cands.push_back({0, kDkWindow, 0});
    if (find_kernel(LT, 0, 1))  // the global-memory kernel (fp64 flushes in either precision)
      for (int k : {4, 8, 16}) cands.push_back({0, 1, k});
    // the untuned default of the class, timed like the others (added when
    // it is not a candidate: the fp64 window kernel serving a mixed context)
    c->tune.erase(LT);
    hfqmc_problem q0 = sample[first];
    q0.delay = 0;
    const Plan def = plan_for(c, q0);
    auto same = [](const Plan& a, const Plan& b) { return a.rt == b.rt && a.dk == b.dk && a.k == b.k; };
    if (std::none_of(cands.begin(), cands.end(), [&](const Plan& x) { return same(x, def); })) cands.push_back(def);
    TuneEntry best{prec_name(c->prec), LT, 0, 0, -1.0, ""};
    TuneEntry dflt = best;
    std::string measured;
    for (const Plan& pl : cands) {
      double tl[2];
      for (int len = 0; len < 2; ++len) {
        const std::vector<hfqmc_problem>& sm = len ? sample2 : sample;
        TRY(stage_impl(c, sm.data(), (int)sm.size(), d_ws, ws_bytes, &pl, true, LT));
        double ms = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
          TRY(enqueue_pass(c, c->stream, true));
          HIP_TRY(hipStreamSynchronize(c->stream));
          double t = 0;  // the class's own launch (its stream's events)
          for (size_t gi = 0; gi < c->groups.size(); ++gi)
            if (c->groups[gi].tuned) {
              float e = 0.f;
              HIP_TRY(hipEventElapsedTime(&e, c->ev[2 * gi], c->ev[2 * gi + 1]));
              t = std::max(t, (double)e);
            }
          if (rep > 0) ms = std::min(ms, t);
        }
        tl[len] = ms;
      }
      // twice the sweeps minus once: the time of `sweeps` sweeps without the
      // fixed costs (the longer run alone if noise made the difference small)
      const double dt = tl[1] - tl[0] > 0.25 * tl[1] ? tl[1] - tl[0] : 0.5 * tl[1];
      const double rate = (double)props / (dt * 1e-3);
      char buf[96];
      std::snprintf(buf, sizeof buf, "%s[%d, %d, %.6g]", measured.empty() ? "" : ", ", pl.rt, pl.k, rate);
      measured += buf;
      if (rate > best.rate) best = {prec_name(c->prec), LT, pl.rt, pl.k, rate, ""};
      if (same(pl, def)) dflt = {prec_name(c->prec), LT, pl.rt, pl.k, rate, ""};
    }
    // shortened chains rank close shapes by noise and by their first sweeps:
    // the default (the best of full-length runs) stays unless a shape beats
    // it by 5 % or more
    if (dflt.rate > 0.0 && best.rate < 1.05 * dflt.rate) best = dflt;
    best.measured = measured;
    c->tune[LT] = best;
    bool replaced = false;
    for (auto& t : c->tune_all)
      if (t.prec == best.prec && t.LT == LT) {
        t = best;
        replaced = true;
      }
    if (!replaced) c->tune_all.push_back(best);
  }
  c->staged = false;  // the workspace now holds the last tuning run
  c->last_launches = 0;
  if (!c->tune_path.empty() && !write_tune_cache(c->tune_path, c->tune_all))
    return fail(HFQMC_EINVAL, "cannot write tune cache %s", c->tune_path.c_str());
  return HFQMC_OK;
}

hfqmc_status hfqmc_plan(hfqmc_ctx* c, int32_t L, int32_t delay, int32_t* rt, int32_t* k, double* tuned_rate) {
  if (!c || L < 1 || L > kMaxL || delay < 0 || delay > kMaxDelay) return fail(HFQMC_EINVAL, "hfqmc_plan: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  hfqmc_problem p{};
  p.L = L;
  p.delay = delay;
  const Plan pl = plan_for(c, p);
  if (rt) *rt = pl.rt;
  if (k) *k = pl.k;
  if (tuned_rate) {
    auto it = c->tune.find(padded_L(L));
    *tuned_rate = it == c->tune.end() ? 0.0 : it->second.rate;
  }
  return HFQMC_OK;
}

// ---------------------------------------------------------------- sites

hfqmc_status hfqmc_attach_pool(hfqmc_ctx* c, void* d_pool, size_t bytes) {
  if (!c || !d_pool || bytes < 4096) return fail(HFQMC_EINVAL, "hfqmc_attach_pool: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!c->sites.empty() || c->srv.started) return fail(HFQMC_EINVAL, "hfqmc_attach_pool: pool in use");
  c->pool = reinterpret_cast<uint8_t*>(d_pool);
  c->pool_bytes = bytes;
  c->free_list.assign(1, PoolBlock{0, bytes / 256 * 256});
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_bytes(int32_t L, int32_t n_bins, int32_t n_chains, size_t* bytes) {
  if (L < 1 || L > kMaxL || n_bins < 2 || n_chains < 0 || n_chains > kMaxChains || !bytes)
    return fail(HFQMC_EINVAL, "hfqmc_site_bytes: bad arguments");
  hfqmc_site s;
  s.L = L;
  s.LT = padded_L(L);
  s.n_bins = n_bins;
  s.n_chains = std::max(1, n_chains);
  *bytes = site_layout(&s);
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_open(hfqmc_ctx* c, int32_t L, int32_t n_bins, int32_t n_chains, hfqmc_site** out) {
  if (!c || !out || L < 1 || L > kMaxL || n_bins < 2 || n_chains < 0 || n_chains > kMaxChains)
    return fail(HFQMC_EINVAL, "hfqmc_site_open: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!c->pool) return fail(HFQMC_EINVAL, "hfqmc_site_open: no pool attached");
  hfqmc_site* s = new (std::nothrow) hfqmc_site;
  if (!s) return fail(HFQMC_ENOMEM, "out of host memory");
  s->L = L;
  hfqmc_problem p{};
  p.L = L;
  p.delay = 0;
  const Plan pl = plan_for(c, p);
  s->LT = pl.LT;
  s->RT = pl.rt;
  s->DK = pl.dk;
  s->K = pl.k;
  s->n_bins = n_bins;
  s->n_chains = std::max(1, n_chains);
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
  if (site_busy(c, s)) return fail(HFQMC_EAGAIN, "site has a serving request in progress");
  pool_free(c, s->off, s->bytes);
  c->sites.erase(it);
  delete s;
  return HFQMC_OK;
}

static hfqmc_status site_upload_problem(hfqmc_ctx* c, hfqmc_site* s, const hfqmc_problem* p, hipStream_t st) {
  uint8_t* base = c->pool + s->off;
  HIP_TRY(hipMemcpyAsync(base + s->o_weiss, p->weiss[0], sizeof(double) * s->L, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(base + s->o_weiss + sizeof(double) * s->L, p->weiss[1], sizeof(double) * s->L,
                         hipMemcpyHostToDevice, st));
  if (p->init_fields) HIP_TRY(hipMemcpyAsync(base + s->o_init, p->init_fields, s->L, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  s->prob = *p;
  s->prob.weiss[0] = s->prob.weiss[1] = nullptr;
  s->prob.init_fields = nullptr;
  s->defined = true;
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_define(hfqmc_ctx* c, hfqmc_site* s, const hfqmc_problem* p) {
  if (!c || !s || !p) return fail(HFQMC_EINVAL, "hfqmc_site_define: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!site_known(c, s)) return fail(HFQMC_ENOTFOUND, "unknown site");
  if (site_busy(c, s)) return fail(HFQMC_EAGAIN, "site has a serving request in progress");
  if (p->L != s->L || p->n_bins != s->n_bins || chains_of(*p) != s->n_chains)
    return fail(HFQMC_EINVAL, "problem L/n_bins/n_chains differ from the site's");
  TRY(validate(*p, 0));
  TRY(set_device(c));
  return site_upload_problem(c, s, p, c->stream);
}

hfqmc_status hfqmc_site_set_fields(hfqmc_ctx* c, hfqmc_site* s, const int8_t* fields) {
  if (!c || !s || !fields) return fail(HFQMC_EINVAL, "hfqmc_site_set_fields: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!site_known(c, s)) return fail(HFQMC_ENOTFOUND, "unknown site");
  if (site_busy(c, s)) return fail(HFQMC_EAGAIN, "site has a serving request in progress");
  if (!s->defined) return fail(HFQMC_EINVAL, "site has no problem (call hfqmc_site_define)");
  for (int k = 0; k < s->L; ++k)
    if (fields[k] != 1 && fields[k] != -1) return fail(HFQMC_EINVAL, "fields[%d] not +-1", k);
  TRY(set_device(c));
  HIP_TRY(hipMemcpyAsync(c->pool + s->off + s->o_init, fields, s->L, hipMemcpyHostToDevice, c->stream));
  ImpDesc d{};
  fill_constants(d, s->prob);
  apply_settings(d, c);
  d.op = OP_FORCE;
  d.n_force = 0;
  d.flags = F_FIELDS_GIVEN | F_SAVE | F_SAVE_G | F_ZERO_ACC;
  for (int j = 0; j < s->n_chains; ++j) TRY(site_launch(c, s, d, j));  // every chain starts here
  s->has_state = true;
  return HFQMC_OK;
}

hfqmc_status hfqmc_site_force_flips(hfqmc_ctx* c, hfqmc_site* s, const int32_t* slices, int32_t n, double* ratios) {
  if (!c || !s || n < 0 || (n > 0 && !slices)) return fail(HFQMC_EINVAL, "hfqmc_site_force_flips: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!site_known(c, s)) return fail(HFQMC_ENOTFOUND, "unknown site");
  if (site_busy(c, s)) return fail(HFQMC_EAGAIN, "site has a serving request in progress");
  if (!s->has_state) return fail(HFQMC_EINVAL, "site has no state (call hfqmc_site_set_fields)");
  for (int k = 0; k < n; ++k)
    if (slices[k] < 0 || slices[k] >= s->L) return fail(HFQMC_EINVAL, "slice %d outside [0,%d)", slices[k], s->L);
  TRY(set_device(c));
  uint8_t* base = c->pool + s->off;
  for (int k0 = 0; k0 < n; k0 += 1024) {
    const int m = std::min(1024, n - k0);
    HIP_TRY(hipMemcpyAsync(base + s->o_force, slices + k0, sizeof(int32_t) * m, hipMemcpyHostToDevice, c->stream));
    ImpDesc d{};
    fill_constants(d, s->prob);
    apply_settings(d, c);
  apply_settings(d, c);
    d.op = OP_FORCE;
    d.n_force = m;
    d.flags = F_RESUME | F_SAVE | F_SAVE_G;
    TRY(site_launch(c, s, d));
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
  if (site_busy(c, s)) return fail(HFQMC_EAGAIN, "site has a serving request in progress");
  if (!s->has_state) return fail(HFQMC_EINVAL, "site has no state");
  TRY(set_device(c));
  ImpDesc d{};
  fill_constants(d, s->prob);
  apply_settings(d, c);
  d.op = OP_RECOMPUTE;
  d.flags = F_RESUME | F_SAVE | F_SAVE_G | F_ZERO_ACC;
  TRY(site_launch(c, s, d));
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
  if (site_busy(c, s)) return fail(HFQMC_EAGAIN, "site has a serving request in progress");
  if (!s->has_state) return fail(HFQMC_EINVAL, "site has no state");
  TRY(set_device(c));
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
  if (site_busy(c, s)) return fail(HFQMC_EAGAIN, "site has a serving request in progress");
  if (!s->has_state) return fail(HFQMC_EINVAL, "site has no state");
  TRY(set_device(c));
  HIP_TRY(hipMemcpyAsync(fields, c->pool + s->off + s->o_fields, s->L, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return HFQMC_OK;
}

// ---------------------------------------------------------------- serving

hfqmc_status hfqmc_serve_config(hfqmc_ctx* c, double step_ms, int64_t quantum_proposals, double capacity_cus) {
  if (!c || !(step_ms > 0) || quantum_proposals < 0 || capacity_cus < 0)
    return fail(HFQMC_EINVAL, "hfqmc_serve_config: bad arguments");
  std::lock_guard<std::mutex> g(c->srv.mu);
  c->srv.step_ms = step_ms;
  c->srv.quantum = quantum_proposals;
  c->srv.capacity = capacity_cus > 0 ? capacity_cus : (double)c->n_cu;
  return HFQMC_OK;
}

hfqmc_status hfqmc_submit(hfqmc_ctx* c, hfqmc_site* s, const hfqmc_problem* p, uint64_t* ticket) {
  if (!c || !s || !p || !ticket) return fail(HFQMC_EINVAL, "hfqmc_submit: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  if (!site_known(c, s)) return fail(HFQMC_ENOTFOUND, "unknown site");
  if (p->L != s->L || p->n_bins != s->n_bins || chains_of(*p) != s->n_chains)
    return fail(HFQMC_EINVAL, "problem L/n_bins/n_chains differ from the site's");
  TRY(validate(*p, 0));
  TRY(srv_start(c));
  Server& S = c->srv;
  {
    std::lock_guard<std::mutex> gs(S.mu);
    if (S.failed) return fail(HFQMC_EDEVICE, "serving engine failed: %s", S.error.c_str());
    if (s->busy) return fail(HFQMC_EAGAIN, "site has a request in progress");
    if (S.pending.size() >= S.max_pending) return fail(HFQMC_EAGAIN, "request queue full");
    s->busy = true;  // no launch touches the site until the request is queued
  }
  const bool had_state = s->has_state;
  if (hfqmc_status st = site_upload_problem(c, s, p, S.io)) {
    std::lock_guard<std::mutex> gs(S.mu);
    s->busy = false;
    return st;
  }
  Request* r = new (std::nothrow) Request;
  if (!r) {
    std::lock_guard<std::mutex> gs(S.mu);
    s->busy = false;
    return fail(HFQMC_ENOMEM, "out of host memory");
  }
  r->site = s;
  r->prob = s->prob;
  for (int j = 0; j < s->n_chains; ++j) r->total.push_back(p->n_warmup + chain_measure(*p, j));
  r->done.assign(s->n_chains, 0);
  r->q.assign(s->n_chains, 0);
  r->given = p->init_fields != nullptr;
  r->keep = !r->given && had_state;
  r->weight = (double)s->n_chains / site_bpc(s);
  {
    std::lock_guard<std::mutex> gs(S.mu);
    r->ticket = S.next_ticket++;
    S.tickets[r->ticket] = r;
    S.pending.push_back(r);
    ++S.submitted;
    *ticket = r->ticket;
  }
  S.cv.notify_all();
  return HFQMC_OK;
}

hfqmc_status hfqmc_poll(hfqmc_ctx* c, uint64_t ticket, hfqmc_result* out) {
  if (!c || !out) return fail(HFQMC_EINVAL, "hfqmc_poll: bad arguments");
  Server& S = c->srv;
  std::lock_guard<std::mutex> gs(S.mu);
  auto it = S.tickets.find(ticket);
  if (it == S.tickets.end() || it->second->cancel) return fail(HFQMC_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  if (r->state != R_DONE) return HFQMC_EAGAIN;
  const int L = r->site->L;
  for (int k = 0; k < 2; ++k) {
    if (out->g[k] && !r->g[k].empty()) std::memcpy(out->g[k], r->g[k].data(), sizeof(double) * (L + 1));
    if (out->g_err[k] && !r->gerr[k].empty()) std::memcpy(out->g_err[k], r->gerr[k].data(), sizeof(double) * (L + 1));
  }
  if (out->bins && !r->bins.empty()) std::memcpy(out->bins, r->bins.data(), sizeof(double) * r->bins.size());
  if (out->final_fields && !r->fields.empty()) std::memcpy(out->final_fields, r->fields.data(), L);
  for (int k = 0; k < 2; ++k) {
    out->n[k] = r->res.n[k];
    out->n_err[k] = r->res.n_err[k];
  }
  out->docc = r->res.docc;
  out->docc_err = r->res.docc_err;
  out->accept_rate = r->res.accept_rate;
  out->max_drift = r->res.max_drift;
  out->proposals = r->res.proposals;
  out->accepts = r->res.accepts;
  out->nonpositive = r->res.nonpositive;
  out->status = r->status;
  const hfqmc_status st = r->status;
  S.tickets.erase(it);
  delete r;
  if (st != HFQMC_OK) return fail(st, "request %llu failed%s%s", (unsigned long long)ticket, S.error.empty() ? "" : ": ",
                                  S.error.c_str());
  return HFQMC_OK;
}

hfqmc_status hfqmc_cancel(hfqmc_ctx* c, uint64_t ticket) {
  if (!c) return fail(HFQMC_EINVAL, "hfqmc_cancel: bad arguments");
  Server& S = c->srv;
  std::lock_guard<std::mutex> gs(S.mu);
  auto it = S.tickets.find(ticket);
  if (it == S.tickets.end() || it->second->cancel) return fail(HFQMC_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  if (r->state == R_PENDING || r->state == R_READY || r->state == R_DONE) {
    if (r->state == R_PENDING) S.pending.erase(std::find(S.pending.begin(), S.pending.end(), r));
    if (r->state == R_READY) {
      S.ready.erase(std::find(S.ready.begin(), S.ready.end(), r));
      S.used -= r->weight;
    }
    if (r->state != R_DONE) {
      r->site->busy = false;
      if (!r->first) r->site->has_state = true;
      ++S.cancelled;
    }
    S.tickets.erase(it);
    delete r;
  } else {
    r->cancel = true;  // in flight: dropped when its launch retires
  }
  return HFQMC_OK;
}

hfqmc_status hfqmc_serve_stats(hfqmc_ctx* c, hfqmc_serve_stats_t* out) {
  if (!c || !out) return fail(HFQMC_EINVAL, "hfqmc_serve_stats: bad arguments");
  Server& S = c->srv;
  std::lock_guard<std::mutex> gs(S.mu);
  out->submitted = S.submitted;
  out->completed = S.completed;
  out->cancelled = S.cancelled;
  out->launches = S.launches;
  out->steps = S.steps;
  out->step_ms_avg = S.steps ? S.step_ms_sum / (double)S.steps : 0.0;
  out->launch_ms_avg = S.launches ? S.kernel_ms_sum / (double)S.launches : 0.0;
  out->pending = (int32_t)S.pending.size();
  int32_t inflight = 0;
  for (const auto& L : S.inflight) inflight += (int32_t)L.items.size();
  out->active = (int32_t)S.ready.size() + inflight;
  out->capacity_used = S.used;
  out->capacity = S.capacity > 0 ? S.capacity : (double)c->n_cu;
  return HFQMC_OK;
}

// ---------------------------------------------------------------- dtau -> 0

// Weighted least squares for O(dtau) = sum_k c_k dtau^(2k), k <= order, by
// Householder QR of the weighted design matrix; errors from (A^T W A)^-1 =
// R^-1 R^-T.
hfqmc_status hfqmc_extrapolate(int32_t n, const double* dtau, const double* value, const double* err, int32_t order,
                               double* coef, double* coef_err) {
  if (n < 1 || !dtau || !value || !coef || order < 0 || order > 3 || n < order + 1)
    return fail(HFQMC_EINVAL, "hfqmc_extrapolate: need n >= order + 1, 0 <= order <= 3");
  const int m = order + 1;
  std::vector<double> A((size_t)n * m), y(n);
  for (int i = 0; i < n; ++i) {
    if (!(dtau[i] > 0) || !std::isfinite(dtau[i]) || !std::isfinite(value[i]))
      return fail(HFQMC_EINVAL, "hfqmc_extrapolate: point %d not finite or dtau <= 0", i);
    double w = 1.0;
    if (err) {
      if (!(err[i] > 0) || !std::isfinite(err[i])) return fail(HFQMC_EINVAL, "hfqmc_extrapolate: err[%d] <= 0", i);
      w = 1.0 / err[i];
    }
    const double x = dtau[i] * dtau[i];
    double p = 1.0;
    for (int k = 0; k < m; ++k, p *= x) A[(size_t)i * m + k] = w * p;
    y[i] = w * value[i];
  }
  // Householder: A = Q R, apply Q^T to y; a column whose remainder after the
  // earlier reflections is rounding-sized relative to its own norm means too
  // few distinct dtau for this order
  std::vector<double> col(m, 0.0);
  for (int k = 0; k < m; ++k)
    for (int i = 0; i < n; ++i) col[k] = std::hypot(col[k], A[(size_t)i * m + k]);
  for (int k = 0; k < m; ++k) {
    double nrm = 0.0;
    for (int i = k; i < n; ++i) nrm = std::hypot(nrm, A[(size_t)i * m + k]);
    if (nrm == 0.0) return fail(HFQMC_EINVAL, "hfqmc_extrapolate: too few distinct dtau for order %d", order);
    const double akk = A[(size_t)k * m + k];
    const double alpha = akk > 0 ? -nrm : nrm;
    std::vector<double> v(n, 0.0);
    v[k] = akk - alpha;
    for (int i = k + 1; i < n; ++i) v[i] = A[(size_t)i * m + k];
    double vv = 0.0;
    for (int i = k; i < n; ++i) vv += v[i] * v[i];
    if (vv > 0.0) {
      for (int j = k; j < m; ++j) {
        double d = 0.0;
        for (int i = k; i < n; ++i) d += v[i] * A[(size_t)i * m + j];
        d = 2.0 * d / vv;
        for (int i = k; i < n; ++i) A[(size_t)i * m + j] -= d * v[i];
      }
      double d = 0.0;
      for (int i = k; i < n; ++i) d += v[i] * y[i];
      d = 2.0 * d / vv;
      for (int i = k; i < n; ++i) y[i] -= d * v[i];
    }
    if (std::fabs(A[(size_t)k * m + k]) <= 1e-10 * col[k])
      return fail(HFQMC_EINVAL, "hfqmc_extrapolate: too few distinct dtau for order %d", order);
  }
  // back substitution R c = Q^T y
  for (int k = m - 1; k >= 0; --k) {
    double s = y[k];
    for (int j = k + 1; j < m; ++j) s -= A[(size_t)k * m + j] * coef[j];
    coef[k] = s / A[(size_t)k * m + k];
  }
  if (coef_err) {
    if (!err) {
      for (int k = 0; k < m; ++k) coef_err[k] = NAN;
    } else {
      // Rinv (upper triangular), covariance = Rinv Rinv^T
      std::vector<double> Ri((size_t)m * m, 0.0);
      for (int j = 0; j < m; ++j) {
        Ri[(size_t)j * m + j] = 1.0 / A[(size_t)j * m + j];
        for (int i = j - 1; i >= 0; --i) {
          double s = 0.0;
          for (int k = i + 1; k <= j; ++k) s += A[(size_t)i * m + k] * Ri[(size_t)k * m + j];
          Ri[(size_t)i * m + j] = -s / A[(size_t)i * m + i];
        }
      }
      for (int k = 0; k < m; ++k) {
        double s = 0.0;
        for (int j = k; j < m; ++j) s += Ri[(size_t)k * m + j] * Ri[(size_t)k * m + j];
        coef_err[k] = std::sqrt(s);
      }
    }
  }
  return HFQMC_OK;
}

// ---------------------------------------------------------------- entropy

hfqmc_status hfqmc_entropy(int32_t n_mu, int32_t n_sites, const double* mu, const double* n_lo, const double* n_hi,
                           double T_lo, double T_hi, double* s) {
  if (n_mu < 2 || n_sites < 1 || !mu || !n_lo || !n_hi || !s || !(T_lo > 0) || !(T_hi > T_lo) ||
      !std::isfinite(T_hi))
    return fail(HFQMC_EINVAL, "hfqmc_entropy: need n_mu >= 2, n_sites >= 1, 0 < T_lo < T_hi");
  for (int k = 0; k < n_mu; ++k) {
    if (!std::isfinite(mu[k]) || (k > 0 && !(mu[k] > mu[k - 1])))
      return fail(HFQMC_EINVAL, "hfqmc_entropy: mu must be finite and strictly ascending (index %d)", k);
    for (int i = 0; i < n_sites; ++i)
      if (!std::isfinite(n_lo[(size_t)k * n_sites + i]) || !std::isfinite(n_hi[(size_t)k * n_sites + i]))
        return fail(HFQMC_EINVAL, "hfqmc_entropy: density (%d,%d) not finite", k, i);
  }
  const double inv = 1.0 / (T_hi - T_lo);
  for (int i = 0; i < n_sites; ++i) {
    double acc = 0.0;
    double prev = (n_hi[i] - n_lo[i]) * inv;
    s[i] = 0.0;
    for (int k = 1; k < n_mu; ++k) {
      const double g = (n_hi[(size_t)k * n_sites + i] - n_lo[(size_t)k * n_sites + i]) * inv;
      acc += (mu[k] - mu[k - 1]) * (g + prev) / 2.0;
      s[(size_t)k * n_sites + i] = acc;
      prev = g;
    }
  }
  return HFQMC_OK;
}

// ---------------------------------------------------------------- lattice

}  // extern "C"

struct hfqmc_lattice {
  hfqmc_ctx* ctx = nullptr;    // the context that created it (its calls take no other)
  int n_sites = 0, layer = 0, n_layers = 0;
  double* d_hop = nullptr;     // caller's memory: n_layers blocks layer x layer, then (n_layers - 1) x layer couplings
  int32_t* d_sites = nullptr;  // caller's memory, after the blocks: n_sites entries for a site list
};

namespace {

size_t lattice_hop_doubles(int N, int b) {
  const int nl = N / b;
  return (size_t)nl * b * b + (size_t)(nl > 1 ? nl - 1 : 0) * b;
}

size_t lattice_mem_bytes(int N, int b) { return align_up(sizeof(double) * lattice_hop_doubles(N, b), 256) + align_up(sizeof(int32_t) * N, 256); }

// Copy a host site list (indices checked, at most n_sites entries) into the
// lattice's device buffer, in stream order after earlier calls that read it;
// returns once the copy is done, so the host list may go at once.
hfqmc_status lattice_sites(hfqmc_ctx* c, hfqmc_lattice* lat, const int32_t* sites, int32_t n_sel) {
  if (n_sel > lat->n_sites) return fail(HFQMC_EINVAL, "site list of %d entries > %d sites", n_sel, lat->n_sites);
  for (int j = 0; j < n_sel; ++j)
    if (sites[j] < 0 || sites[j] >= lat->n_sites)
      return fail(HFQMC_EINVAL, "site %d of the list (%d) outside [0,%d)", j, sites[j], lat->n_sites);
  HIP_TRY(hipMemcpyAsync(lat->d_sites, sites, sizeof(int32_t) * n_sel, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return HFQMC_OK;
}

}  // namespace

extern "C" {

hfqmc_status hfqmc_lattice_bytes(int32_t n_sites, int32_t layer, size_t* bytes) {
  if (!bytes || layer < 1 || layer > kMaxLayer || n_sites < layer || n_sites % layer)
    return fail(HFQMC_EINVAL, "hfqmc_lattice_bytes: need 1 <= layer <= %d dividing n_sites", kMaxLayer);
  *bytes = lattice_mem_bytes(n_sites, layer);
  return HFQMC_OK;
}

hfqmc_status hfqmc_lattice_create(hfqmc_ctx* c, int32_t n_sites, int32_t layer, const double* hop, void* d_mem,
                                  size_t mem_bytes, hfqmc_lattice** out) {
  if (!c || !hop || !out || !d_mem || layer < 1 || layer > kMaxLayer || n_sites < layer || n_sites % layer)
    return fail(HFQMC_EINVAL, "hfqmc_lattice_create: need 1 <= layer <= %d dividing n_sites", kMaxLayer);
  if (mem_bytes < lattice_mem_bytes(n_sites, layer))
    return fail(HFQMC_ENOMEM, "lattice memory %zu bytes < %zu needed", mem_bytes, lattice_mem_bytes(n_sites, layer));
  const int N = n_sites, b = layer, nl = N / b;
  double scale = 0.0;
  for (size_t k = 0; k < (size_t)N * N; ++k) {
    if (!std::isfinite(hop[k])) return fail(HFQMC_EINVAL, "hop[%zu] not finite", k);
    scale = std::max(scale, std::fabs(hop[k]));
  }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const double h = hop[(size_t)i * N + j];
      if (std::fabs(h - hop[(size_t)j * N + i]) > 1e-14 * scale)
        return fail(HFQMC_EINVAL, "hop not symmetric at (%d,%d)", i, j);
      const int li = i / b, lj = j / b;
      const bool allowed = li == lj || (std::abs(li - lj) == 1 && i % b == j % b);
      if (h != 0.0 && !allowed)
        return fail(HFQMC_EINVAL,
                    "hop(%d,%d) = %g: only hopping inside a layer of %d sites or between the same position of "
                    "neighbouring layers is supported", i, j, h, b);
    }
  std::vector<double> img((size_t)nl * b * b + (size_t)(nl > 1 ? nl - 1 : 0) * b);
  for (int k = 0; k < nl; ++k)
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < b; ++j) img[((size_t)k * b + i) * b + j] = hop[(size_t)(k * b + i) * N + k * b + j];
  for (int k = 0; k + 1 < nl; ++k)
    for (int j = 0; j < b; ++j) img[(size_t)nl * b * b + (size_t)k * b + j] = hop[(size_t)(k * b + j) * N + (k + 1) * b + j];
  std::lock_guard<std::mutex> g(c->mu);
  TRY(set_device(c));
  hfqmc_lattice* lat = new (std::nothrow) hfqmc_lattice;
  if (!lat) return fail(HFQMC_ENOMEM, "out of host memory");
  lat->ctx = c;
  lat->n_sites = N;
  lat->layer = b;
  lat->n_layers = nl;
  lat->d_hop = reinterpret_cast<double*>(d_mem);
  lat->d_sites = reinterpret_cast<int32_t*>(reinterpret_cast<uint8_t*>(d_mem) +
                                            align_up(sizeof(double) * lattice_hop_doubles(N, b), 256));
  hipError_t e = hipMemcpyAsync(lat->d_hop, img.data(), sizeof(double) * img.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    delete lat;
    return fail(HFQMC_EDEVICE, "hfqmc_lattice_create: %s", hipGetErrorString(e));
  }
  *out = lat;
  return HFQMC_OK;
}

hfqmc_status hfqmc_lattice_destroy(hfqmc_ctx* c, hfqmc_lattice* lat) {
  if (!c || !lat || lat->ctx != c) return fail(HFQMC_EINVAL, "hfqmc_lattice_destroy: bad arguments");
  std::lock_guard<std::mutex> g(c->mu);
  TRY(set_device(c));
  HIP_TRY(hipStreamSynchronize(c->stream));  // calls in flight may still read the caller's lattice memory
  delete lat;
  return HFQMC_OK;
}

hfqmc_status hfqmc_lattice_workspace(const hfqmc_lattice* lat, int32_t n_freq, size_t* bytes) {
  if (!lat || !bytes || n_freq < 1 || n_freq > kMaxFreq)
    return fail(HFQMC_EINVAL, "hfqmc_lattice_workspace: need 1 <= n_freq <= %d", kMaxFreq);
  *bytes = lattice_work_bytes(lat->layer, lat->n_layers, n_freq);
  return HFQMC_OK;
}

hfqmc_status hfqmc_lattice_green(hfqmc_ctx* c, hfqmc_lattice* lat, int32_t n_freq, double beta, double mu,
                                 const double* d_eps, const double* d_sigma, double* d_gloc, void* d_ws,
                                 size_t ws_bytes) {
  if (!c || !lat || !d_eps || !d_sigma || !d_gloc || !d_ws || n_freq < 1 || n_freq > kMaxFreq || !(beta > 0) ||
      !std::isfinite(beta) || !std::isfinite(mu))
    return fail(HFQMC_EINVAL, "hfqmc_lattice_green: bad arguments");
  if (lat->ctx != c) return fail(HFQMC_EINVAL, "hfqmc_lattice_green: lattice of another context");
  const size_t need = lattice_work_bytes(lat->layer, lat->n_layers, n_freq);
  if (ws_bytes < need) return fail(HFQMC_ENOMEM, "lattice workspace %zu bytes < %zu needed", ws_bytes, need);
  std::lock_guard<std::mutex> g(c->mu);
  TRY(set_device(c));
  LatDesc d{};
  d.n_sites = lat->n_sites;
  d.layer = lat->layer;
  d.n_layers = lat->n_layers;
  d.n_freq = n_freq;
  d.beta = beta;
  d.mu = mu;
  d.blocks = lat->d_hop;
  d.coupling = lat->d_hop + (size_t)lat->n_layers * lat->layer * lat->layer;
  d.eps = d_eps;
  d.sigma = d_sigma;
  d.gloc = d_gloc;
  d.work = reinterpret_cast<double*>(d_ws);
  HIP_TRY(launch_lattice_green(d, c->stream));
  return HFQMC_OK;
}

hfqmc_status hfqmc_lattice_weiss(hfqmc_ctx* c, hfqmc_lattice* lat, int32_t n_freq, double beta, double mu, int32_t L,
                                 const double* d_eps, const double* d_gloc, const double* d_sigma,
                                 const int32_t* sites, int32_t n_sel, double* d_weiss_iw, double* d_weiss_tau) {
  if (!c || !lat || !d_eps || !d_gloc || !d_sigma || !sites || !d_weiss_iw || !d_weiss_tau || n_sel < 1 ||
      n_freq < 1 || n_freq > kMaxFreq || L < 2 || L > kMaxL || !(beta > 0) || !std::isfinite(beta) ||
      !std::isfinite(mu))
    return fail(HFQMC_EINVAL, "hfqmc_lattice_weiss: bad arguments");
  if (lat->ctx != c) return fail(HFQMC_EINVAL, "hfqmc_lattice_weiss: lattice of another context");
  std::lock_guard<std::mutex> g(c->mu);
  TRY(set_device(c));
  TRY(lattice_sites(c, lat, sites, n_sel));
  WeissDesc d{};
  d.n_sites = lat->n_sites;
  d.n_freq = n_freq;
  d.L = L;
  d.n_sel = n_sel;
  d.beta = beta;
  d.mu = mu;
  d.eps = d_eps;
  d.gloc = d_gloc;
  d.sigma = d_sigma;
  d.sites = lat->d_sites;
  d.weiss_iw = d_weiss_iw;
  d.weiss_tau = d_weiss_tau;
  HIP_TRY(launch_weiss(d, c->stream));
  return HFQMC_OK;
}

hfqmc_status hfqmc_lattice_sigma(hfqmc_ctx* c, hfqmc_lattice* lat, int32_t n_freq, double beta, double mu, double U,
                                 int32_t L, const double* d_eps, const int32_t* sites, int32_t n_sel,
                                 const double* d_weiss_iw, const double* d_gimp_tau, const double* d_density,
                                 double mix, double* d_sigma) {
  if (!c || !lat || !d_eps || !sites || !d_weiss_iw || !d_gimp_tau || !d_density || !d_sigma || n_sel < 1 ||
      n_freq < 1 || n_freq > kMaxFreq || L < 2 || L > kMaxL || !(beta > 0) || !std::isfinite(beta) ||
      !std::isfinite(mu) || !(U >= 0) || !std::isfinite(U) || !(mix > 0 && mix <= 1))
    return fail(HFQMC_EINVAL, "hfqmc_lattice_sigma: bad arguments");
  if (lat->ctx != c) return fail(HFQMC_EINVAL, "hfqmc_lattice_sigma: lattice of another context");
  std::vector<int32_t> sorted(sites, sites + n_sel);
  std::sort(sorted.begin(), sorted.end());
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
    return fail(HFQMC_EINVAL, "hfqmc_lattice_sigma: a site appears twice in the list");
  std::lock_guard<std::mutex> g(c->mu);
  TRY(set_device(c));
  TRY(lattice_sites(c, lat, sites, n_sel));
  SigmaDesc d{};
  d.n_sites = lat->n_sites;
  d.n_freq = n_freq;
  d.L = L;
  d.n_sel = n_sel;
  d.beta = beta;
  d.mu = mu;
  d.U = U;
  d.mix = mix;
  d.eps = d_eps;
  d.sites = lat->d_sites;
  d.weiss_iw = d_weiss_iw;
  d.gimp_tau = d_gimp_tau;
  d.density = d_density;
  d.sigma = d_sigma;
  HIP_TRY(launch_sigma(d, c->stream));
  return HFQMC_OK;
}

}  // extern "C"
