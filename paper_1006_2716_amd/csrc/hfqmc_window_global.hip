// hfqmc_window_global.hip -- window (submatrix) updates for imaginary-time
// grids whose two L x L Green matrices live in device memory (L > 128).
//
// The chain is the one of every other kernel: Metropolis test of
// R = R_up R_dn, R_s = 1 + (1 - G_s[l][l]) d_s (Eq. (1) and the ratio of the
// "Model and Methods" section), flips accepted with probability min(1, R),
// from-scratch Dyson solves G = [1 + (1 - G0)(e^V - 1)]^{-1} G0 (Eq. (2)).
// The slices of a sweep are taken in windows W of 16: wave 0 decides the
// whole window on the two 16 x 16 diagonal blocks G_s[W,W] in registers
// (hfqmc_wscan.h), and the window's accepts S then reach all of G as one
// rank-|S| product
//     G_s += (G_s[:,S] - E_S) P_s G_s[S,:],   P_s = (D_s Q_s)[S,S],
// on the matrix cores (v_mfma_f64_16x16x4f64).  G_s stays row-major in the
// impurity's state area (resident in L2 / the last-level cache while the
// workgroup runs); per window the workgroup stages the window's column
// strip G_s[:,W] and row strip G_s[W,:] in LDS, and wave w streams tile-row
// w of both spins through its registers once.  Compared with per-accept
// delayed updates this removes the strided column gather of every accept:
// G moves through the CU once per window, not once per k accepts, and the
// decisions of a window need no memory traffic at all.
#include "hfqmc_wscan.h"

namespace hfqmc {

template <int LT_>
struct GWCfg {
  static constexpr int LT = LT_;
  static constexpr int NT = LT / 16;         // tiles per dimension = windows per sweep
  static constexpr int NW = NT;              // wave w: tile-row w of both spins
  static constexpr int NTH = 64 * NW;
  static constexpr int JW = (LT + 63) / 64;  // 64-slice words of the field masks
  static constexpr int CS = 17;              // row stride of the column strip and of P
  static constexpr int RSS = LT + 2;         // row stride of the row strip
  static constexpr int RB = 64;              // rows of G per measurement block
  static_assert(LT % 16 == 0 && NTH >= 2 * LT, "bad configuration");
};

template <class C>
struct GWSmem {
  union {
    struct {
      double cs[2][C::LT * C::CS];  // column strip G_s[:,W] (rows CS apart)
      double rs[2][16 * C::RSS];    // row strip G_s[W,:]
    } w;
    double rows[C::RB * C::LT];     // a block of rows of G_s for the g(tau) estimator
  } u;
  double pb[2][16 * C::CS];         // P_s of the window (window coordinates)
  double weiss[2][C::LT];
  double red[C::NW];
  uint32_t win[4];                  // S, |S| (+ bad bit), accepted slices (4 bits each)
  int item;
};

template <class C>
struct EngineGW {
  static constexpr int LT = C::LT, NT = C::NT, JW = C::JW, CS = C::CS, RSS = C::RSS;
  static constexpr int CH = NT;  // tiles per chunk of the flush: a whole tile-row in flight

  GWSmem<C>& sm;
  // thread and wave indices; refresh_ids() re-derives them behind an opaque
  // asm statement at the start of every window and measurement, so the
  // addresses built from them are recomputed there instead of hoisted out of
  // the sweep loop into long-lived registers (hoisted, they pushed the wave-0
  // scan into scratch: 168 VGPRs + 97 spilled, now 128 and none)
  int tid, wave, lane, q, c;
  uint64_t fm[JW];          // fields: bit set <=> s = -1 (uniform)
  int L = 0;
  ImpDesc d;
  gdouble* gm = nullptr;    // G_up, G_dn (LT x LT each, row-major), then the drift snapshot
  int64_t accepts = 0, nonpos = 0, err = 0;  // wave-0 counters
  double px = 1.0;          // test hook: NaN poisons the blocks the sweep's decisions read

  __device__ __forceinline__ EngineGW(GWSmem<C>& s)
      : sm(s),
        tid(threadIdx.x),
        wave(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)),
        lane(threadIdx.x & 63),
        q((threadIdx.x & 63) >> 4),
        c(threadIdx.x & 15) {}

  // Stores of every wave to G visible to the loads of every wave: the
  // workgroup-scope release/acquire of the barrier suffices (the waves share
  // the CU's caches); a device-scope fence would write back and invalidate
  // the whole L2 each time.
  __device__ __forceinline__ void publish() { __syncthreads(); }

  __device__ __forceinline__ void refresh_ids() {
    int t = threadIdx.x;
    __asm__ volatile("" : "+v"(t));
    tid = t;
    lane = t & 63;
    q = (t >> 4) & 3;
    c = t & 15;
    int w = __builtin_amdgcn_readfirstlane(t >> 6);
    __asm__ volatile("" : "+s"(w));
    wave = w;
  }

  __device__ __forceinline__ gdouble* gs(int s) const { return gm + (size_t)s * LT * LT; }

  // x where c holds, else 0, as a product: with a select the compiler moves
  // the load of x into a branch that waits for its own round trip (x is
  // finite: an element of P or of the staged strips)
  __device__ __forceinline__ static double keep(bool c, double x) { return x * (c ? 1.0 : 0.0); }

  // G = G0 of both spins: the antiperiodic matrix of the Weiss samples.
  __device__ __forceinline__ void set_weiss() {
    for (int idx = tid; idx < 2 * LT * LT; idx += C::NTH) {
      const int s = idx / (LT * LT), i = (idx / LT) % LT, j = idx % LT;
      double v = 0.0;
      if (i < L && j < L) v = i >= j ? sm.weiss[s][i - j] : -sm.weiss[s][i - j + L];
      gm[idx] = v;
    }
    publish();
  }

  // The diagonal 16 x 16 tiles of both spins, parked behind G (drift of the
  // next Dyson solve).
  __device__ __forceinline__ void save_diag_tiles() {
    gdouble* snap = gm + 2 * (size_t)LT * LT;
    for (int idx = tid; idx < 2 * NT * 256; idx += C::NTH) {
      const int s = idx / (NT * 256), t = (idx / 256) % NT, i = (idx / 16) & 15, j = idx & 15;
      snap[idx] = gs(s)[(size_t)(16 * t + i) * LT + 16 * t + j];
    }
    __syncthreads();  // read before G is overwritten
  }

  // max |G_parked - G| over the diagonal tiles (uniform).
  __device__ __forceinline__ double diag_tile_drift() {
    const gdouble* snap = gm + 2 * (size_t)LT * LT;
    double dr = 0.0;
    for (int idx = tid; idx < 2 * NT * 256; idx += C::NTH) {
      const int s = idx / (NT * 256), t = (idx / 256) % NT, i = (idx / 16) & 15, j = idx & 15;
      dr = fmax(dr, fabs(snap[idx] - gs(s)[(size_t)(16 * t + i) * LT + 16 * t + j]));
    }
    dr = wave_max(dr);
    if (lane == 0) sm.red[wave] = dr;
    __syncthreads();
    dr = 0.0;
    for (int w = 0; w < C::NW; ++w) dr = fmax(dr, sm.red[w]);
    __syncthreads();
    return dr;
  }

  // Column strip G_s[:,W] and row strip G_s[W,:] of window ww into LDS.
  // With 64 threads per tile-row, a strip of one spin is exactly four
  // elements per thread at compile-time offsets; every load of a thread is
  // issued before its first LDS store (a loop of load-then-store pairs would
  // wait one memory round trip per element).
  static_assert(16 * C::LT == 4 * C::NTH, "one tile-row per wave");
  __device__ __forceinline__ void stage_strips(int ww) {
    const int base = 16 * ww;
    constexpr int RSTEP = C::NTH / 16;  // column-strip rows per step
    const int ci = tid >> 4, cj = tid & 15;            // column strip: row ci + RSTEP v, column cj
    const int ri = tid / LT, rj = tid - (tid / LT) * LT;  // row strip: row ri + 4 v, column rj
    const gdouble* pc = gm + (size_t)ci * LT + base + cj;
    const gdouble* pr = gm + (size_t)(base + ri) * LT + rj;
    double vc[2][4], vr[2][4];
    static_for<2>([&](auto s) __attribute__((always_inline)) {
      static_for<4>([&](auto v) __attribute__((always_inline)) {
        vc[s][v] = pc[(size_t)s * LT * LT + (size_t)v * RSTEP * LT];
        vr[s][v] = pr[(size_t)s * LT * LT + (size_t)v * 4 * LT];
      });
    });
    static_for<2>([&](auto s) __attribute__((always_inline)) {
      static_for<4>([&](auto v) __attribute__((always_inline)) {
        sm.u.w.cs[s][(ci + v * RSTEP) * CS + cj] = vc[s][v];
        sm.u.w.rs[s][(ri + 4 * v) * RSS + rj] = vr[s][v];
      });
    });
    __syncthreads();
  }

  // Wave 0: the window's decisions on the diagonal blocks of the staged
  // column strip.
  __device__ __forceinline__ void scan(int ww, int mode, int jf, const uint64_t (&xw)[JW], double* ratio_out) {
    const int base = 16 * ww;
    const uint32_t fw0 = (uint32_t)(pick<JW>(fm, base >> 6) >> (base & 63)) & 0xFFFFu;
    const double fa = mode == WM_DYSON ? +d.dset_p : +d.dflip_p;  // sigma s_l = +1
    const double fb = mode == WM_DYSON ? +d.dset_m : +d.dflip_m;  // sigma s_l = -1
    double u = 0.0;
    if (mode == WM_METROPOLIS) u = bperm_d(((base + c) & 63) << 2, u01(pick<JW>(xw, ww >> 2)));
    win_scan<CS>(sm.u.w.cs[0] + (base + 4 * q) * CS + c, sm.u.w.cs[1] + (base + 4 * q) * CS + c, CS, lane, q, c,
                 base, L, fw0, fa, fb, mode, jf, u, px, ratio_out, sm.pb[0], sm.pb[1], sm.win, accepts, nonpos, err);
  }

  // Wave w, tile-row w of spin s: V = P_s^T (G_s[rows, S] - E)^T, then for
  // every tile column G_s[rows, tj] += V^T G_s[S, tj] (fp64 accumulator rows
  // fed permuted so that it lands in the layout lane (q, c), register r =
  // row 4q + r, column c), tile by tile from and back to device memory.
  // The ceil(|S| / 4) matrix-core steps of a tile run as a loop over the
  // groups of four accepted slices: one code path for every |S| (a branch
  // per group count, each unrolled, spilled 150 registers per lane here).
  __device__ __forceinline__ void flush(int ww, int m, uint64_t slist) {
    const int ii = lane & 15, qq = lane >> 4;
    const int si = (int)(slist >> (4 * ii)) & 15;
    const int K4 = (m + 3) >> 2;
    const int pi = 4 * (ii & 3) + (ii >> 2);
    const int ti = wave;
    for (int s = 0; s < 2; ++s) {
      const double* pb = sm.pb[s];
      const double* cs = sm.u.w.cs[s];
      const double* rs = sm.u.w.rs[s];
      gdouble* g = gs(s) + (size_t)(16 * ti + 4 * q) * LT + c;
      __asm__ volatile("" : "+v"(g));  // addresses derived here, not hoisted out of the spin loop
      wd4 V = {0.0, 0.0, 0.0, 0.0};
      for (int gi = 0; gi < K4; ++gi) {
        const int k = 4 * gi + qq;
        const bool kv = k < m;
        const int sk = (int)(slist >> (4 * k)) & 15;
        const double x = pb[sk * CS + si];
        const double y = cs[(16 * ti + pi) * CS + sk] - ((ti == ww && pi == sk) ? 1.0 : 0.0);
        V = __builtin_amdgcn_mfma_f64_16x16x4f64(keep(kv && ii < m, x), keep(kv, y), V, 0, 0, 0);
      }
      // chunks of CH tiles: all loads of a chunk are in flight together
      static_for<(NT + CH - 1) / CH>([&](auto ch) __attribute__((always_inline)) {
        constexpr int T0 = decltype(ch)::value * CH;
        constexpr int TN = NT - T0 < CH ? NT - T0 : CH;
        gdouble* gc = g + 16 * T0;
        __asm__ volatile("" : "+v"(gc));
        wd4 acc[TN];
        static_for<TN>([&](auto u) __attribute__((always_inline)) {
          static_for<4>([&](auto r) __attribute__((always_inline)) {
            acc[u][decltype(r)::value] = gc[(size_t)r * LT + 16 * u];
          });
        });
        for (int gi = 0; gi < K4; ++gi) {
          const int k = 4 * gi + qq;
          const bool kv = k < m;
          const int sk = (int)(slist >> (4 * k)) & 15;
          const double a = gi == 0 ? V[0] : gi == 1 ? V[1] : gi == 2 ? V[2] : V[3];
          static_for<TN>([&](auto u) __attribute__((always_inline)) {
            const double x = rs[sk * RSS + 16 * (T0 + u) + ii];
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, keep(kv, x), acc[u], 0, 0, 0);
          });
        }
        static_for<TN>([&](auto u) __attribute__((always_inline)) {
          static_for<4>([&](auto r) __attribute__((always_inline)) {
            gc[(size_t)r * LT + 16 * u] = acc[u][decltype(r)::value];
          });
        });
      });
    }
  }

  // One window on every wave.  Returns 1 if a ratio of the window's scan was
  // not a positive number (the same on every thread), else 0.
  __device__ __forceinline__ uint32_t window(int ww, int mode, int jf, const uint64_t (&xw)[JW], double* ratio_out) {
    refresh_ids();
    stage_strips(ww);
    if (wave == 0) scan(ww, mode, jf, xw, ratio_out);
    __syncthreads();
    const uint32_t S = __builtin_amdgcn_readfirstlane(sm.win[0]);
    const uint32_t w1 = __builtin_amdgcn_readfirstlane(sm.win[1]);
    const int m = (int)(w1 & 0xFFu);
    const uint64_t slist = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(sm.win[2]) |
                           ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(sm.win[3]) << 32);
    if (mode != WM_DYSON && S) {
      const int base = 16 * ww;
      static_for<JW>([&](auto jj) __attribute__((always_inline)) {
        if (jj == (base >> 6)) fm[jj] ^= (uint64_t)S << (base & 63);
      });
    }
    if (m) {
      flush(ww, m, slist);
      publish();  // the next window stages the updated strips
    }
    return (w1 >> 8) & 1u;
  }

  // n consecutive doubles from device memory into the row buffer, all loads
  // of a thread in flight before its first store.
  static constexpr int NR = (C::RB * LT + C::NTH - 1) / C::NTH;
  __device__ __forceinline__ void stage_rows(const gdouble* src, int n) {
    double v[NR];
    static_for<NR>([&](auto u) __attribute__((always_inline)) {
      const int idx = tid + u * C::NTH;
      v[u] = idx < n ? src[idx] : 0.0;
    });
    static_for<NR>([&](auto u) __attribute__((always_inline)) {
      const int idx = tid + u * C::NTH;
      if (idx < n) sm.u.rows[idx] = v[u];
    });
  }

  // g_s(tau_k) sums S_k = sum_l eps G_s[(l+k) mod L][l], staged through LDS
  // in blocks of rows; thread t = s*L + k returns S_k / L.
  __device__ __forceinline__ double green_sums() {
    refresh_ids();
    const int sme = tid >= L, k = tid - sme * L;
    double S = 0.0;
    for (int s = 0; s < 2; ++s) {
      const gdouble* Gs = gs(s);
      for (int r0 = 0; r0 < L; r0 += C::RB) {
        const int r1 = r0 + C::RB < L ? r0 + C::RB : L;
        __syncthreads();
        stage_rows(Gs + (size_t)r0 * LT, (r1 - r0) * LT);
        __syncthreads();
        if (tid < 2 * L && sme == s) {
          const double* R = sm.u.rows;
          int lo = r0 - k > 0 ? r0 - k : 0, hi = (L - k) < (r1 - k) ? (L - k) : (r1 - k);
          for (int l = lo; l < hi; ++l) S += R[(l + k - r0) * LT + l];      // row l + k
          lo = (L - k) > (r0 - k + L) ? (L - k) : (r0 - k + L);
          hi = L < (r1 - k + L) ? L : (r1 - k + L);
          for (int l = lo; l < hi; ++l) S -= R[(l + k - L - r0) * LT + l];  // row l + k - L
        }
      }
    }
    __syncthreads();  // the strips reuse the row buffer
    return S / (double)L;
  }

  __device__ __forceinline__ void run(const ImpDesc* desc, uint8_t* ws) {
    d = *desc;
    L = d.L;
    accepts = nonpos = err = 0;
    gm = (gdouble*)(ws + d.off_state);  // the workspace is device memory
    const int flags = d.flags;
    const int NV = n_values(L);
    double* bins = reinterpret_cast<double*>(ws + d.off_bins);
    ImpStatus* st = reinterpret_cast<ImpStatus*>(ws + d.off_status);
    int8_t* fields = reinterpret_cast<int8_t*>(ws + d.off_fields);
    const double* wv = reinterpret_cast<const double*>(ws + d.off_weiss);
    const int32_t* fslices = reinterpret_cast<const int32_t*>(ws + d.off_force);
    double* fratios = reinterpret_cast<double*>(ws + d.off_force + 4 * ((d.n_force + 1) & ~1));

    if (flags & F_ZERO_ACC) {
      for (int i = tid; i < d.n_bins * NV; i += C::NTH) bins[i] = 0.0;
      if (tid == 0) {
        st->proposals = st->accepts = st->nonpositive = st->error = 0;
        st->max_drift = 0.0;
        st->recoveries = 0;
      }
    }
    // recompute schedule: every recompute_every sweeps, or with a drift limit
    // the (possibly shortened) schedule a previous launch of the chain left
    int64_t next_rec = d.sweep_begin + (d.recompute_every - 1 - d.sweep_begin % d.recompute_every);
    int rec_every = d.recompute_every;
    if (d.drift_limit > 0.0 && !(flags & F_ZERO_ACC) && st->rec_every > 0) {
      next_rec = st->next_rec;
      rec_every = st->rec_every;
    }
    for (int i = tid; i < 2 * LT; i += C::NTH) {
      const int s = i / LT, k = i % LT;
      sm.weiss[s][k] = k < L ? wv[s * L + k] : 0.0;
    }
    if (flags & (F_FIELDS_GIVEN | F_RESUME | F_KEEP_FIELDS)) {
      const int8_t* fin = (flags & F_FIELDS_GIVEN) ? reinterpret_cast<const int8_t*>(ws + d.off_init) : fields;
      static_for<JW>([&](auto jj) __attribute__((always_inline)) {
        const int m = lane + 64 * jj;
        fm[jj] = __ballot(m < L && fin[m] < 0);
      });
    } else {
      const U64x4 x = philox4x64_10((uint64_t)lane, 0, kPurposeInit, (uint64_t)d.chain, d.seed, d.site);
      static_for<JW>([&](auto jj) __attribute__((always_inline)) {
        const int m = lane + 64 * jj;
        fm[jj] = __ballot(m < L && (x.v[jj] >> 63));
      });
    }
    __syncthreads();

    const bool sweeps = d.op == OP_SWEEPS;
    const int64_t nm = d.n_measure, nb = d.n_bins;
    // running bin sums, loaded on entry to a bin and stored when it is left
    // or the launch ends (a chain split over launches sums like one launch)
    double gacc = 0.0, nacc_u = 0.0, nacc_d = 0.0, dacc = 0.0;
    int64_t cur_bin = -1;
    int64_t proposals = 0;
    double max_drift = 0.0;
    // numeric recovery: a sweep whose scan saw a ratio that was not a
    // positive number is repeated once, from its starting fields and a
    // from-scratch Dyson solve; the repeat failing too leaves the error set
    int attempt = 0, recoveries = 0;
    uint64_t fm0[JW];
    int64_t acc0 = 0, np0 = 0, err0 = 0;

    int64_t w = d.sweep_begin;  // sweep of the next Metropolis pass
    int kf = 0;                 // next forced flip
    int mode = (flags & F_RESUME) ? WM_METROPOLIS : WM_DYSON;
    bool drift = false;
    bool measure_after = false;
    if (d.op == OP_RECOMPUTE) {
      mode = WM_DYSON;
      drift = (flags & F_RESUME) != 0;
    }
    for (;;) {
      if (mode == WM_METROPOLIS) {
        if (d.op == OP_FORCE) {
          if (kf >= d.n_force) break;
          mode = WM_FORCE;
        } else if (!sweeps || w >= d.sweep_end) {
          break;
        }
      }
      int ww0 = 0, ww1 = (L + 15) >> 4, jf = 0;
      double* rout = nullptr;
      px = 1.0;
      uint64_t xw[JW];
      static_for<JW>([&](auto jj) __attribute__((always_inline)) { xw[jj] = 0; });
      if (mode == WM_DYSON) {
        if (drift) save_diag_tiles();
        set_weiss();
      } else if (mode == WM_FORCE) {
        const int l = fslices[kf];
        ww0 = l >> 4;
        ww1 = ww0 + 1;
        jf = l & 15;
        rout = fratios + kf;
      } else {
        static_for<JW>([&](auto jj) __attribute__((always_inline)) { fm0[jj] = fm[jj]; });
        acc0 = accepts;
        np0 = nonpos;
        err0 = err;
        px = (attempt ? +d.poison[1] : +d.poison[0]) == w + 1 ? __builtin_nan("") : 1.0;
        if (wave == 0) {
          const U64x4 x = philox4x64_10((uint64_t)lane, (uint64_t)(w + d.rng_offset), kPurposeSweep,
                                        (uint64_t)d.chain, d.seed, d.site);
          static_for<JW>([&](auto jj) __attribute__((always_inline)) { xw[jj] = x.v[jj]; });
        }
      }
      uint32_t bad = 0;
      for (int ww = ww0; ww < ww1; ++ww) bad |= window(ww, mode, jf, xw, rout);
      bool measure = false;
      if (mode == WM_DYSON) {
        if (drift) {
          const double dr = diag_tile_drift();
          max_drift = fmax(max_drift, dr);
          if (d.op != OP_RECOMPUTE) {
            if (d.drift_limit > 0.0 && !(dr <= d.drift_limit)) {
              if (rec_every > 1)
                rec_every >>= 1;
              else
                err = 1;
            }
            next_rec += rec_every;
          }
        }
        if (d.op == OP_RECOMPUTE) break;
        measure = measure_after;
        measure_after = false;
        mode = WM_METROPOLIS;
      } else if (mode == WM_FORCE) {
        ++kf;
        mode = WM_METROPOLIS;
      } else if (bad && attempt == 0) {  // repeat sweep w from a Dyson solve
        static_for<JW>([&](auto jj) __attribute__((always_inline)) { fm[jj] = fm0[jj]; });
        accepts = acc0;
        nonpos = np0;
        err = err0;
        attempt = 1;
        ++recoveries;
        mode = WM_DYSON;
        drift = false;
        measure_after = false;
        continue;
      } else {
        attempt = 0;
        proposals += L;
        ++w;
        if (w - 1 == next_rec) {  // recompute first, then measure sweep w - 1
          mode = WM_DYSON;
          drift = true;
          measure_after = true;
        } else {
          measure = true;
        }
      }
      if (!measure || w - 1 < d.n_warmup) continue;
      // ---- measurement of sweep w - 1
      const int64_t m = w - 1 - d.n_warmup;
      const int64_t b = (m * nb) / nm;
      double* bp = bins + (size_t)b * NV;
      if (b != cur_bin) {
        gacc = tid < 2 * L ? bp[tid + (tid >= L)] : 0.0;
        nacc_u = bp[2 * L + 2];
        nacc_d = bp[2 * L + 3];
        dacc = bp[2 * L + 4];
        cur_bin = b;
      }
      {
        double xu = 0.0, xd = 0.0, xx = 0.0;
        static_for<JW>([&](auto jj) __attribute__((always_inline)) {
          const int mm = lane + 64 * jj;
          if (mm < L) {
            const double u1 = 1.0 - gs(0)[(size_t)mm * LT + mm], d1 = 1.0 - gs(1)[(size_t)mm * LT + mm];
            xu += u1;
            xd += d1;
            xx += u1 * d1;
          }
        });
        nacc_u += wave_sum(xu) / (double)L;
        nacc_d += wave_sum(xd) / (double)L;
        dacc += wave_sum(xx) / (double)L;
      }
      const double gk = green_sums();
      if (tid < 2 * L) gacc += gk;
      const bool last = (m + 1 == nm) || (((m + 1) * nb) / nm != b) || (w == d.sweep_end);
      if (last) {
        if (tid < 2 * L) bp[tid + (tid >= L)] = gacc;
        if (tid == 0) {
          bp[L] = nacc_u;
          bp[2 * L + 1] = nacc_d;
          bp[2 * L + 2] = nacc_u;
          bp[2 * L + 3] = nacc_d;
          bp[2 * L + 4] = dacc;
        }
        cur_bin = -1;
      }
    }

    if ((flags & F_SAVE) && wave == 0) {  // G is already in its state area
      static_for<JW>([&](auto jj) __attribute__((always_inline)) {
        const int m = lane + 64 * jj;
        if (m < L) fields[m] = ((fm[jj] >> lane) & 1) ? (int8_t)-1 : (int8_t)1;
      });
    }
    if (tid == 0) {
      st->proposals += proposals;
      st->accepts += accepts;
      st->nonpositive += nonpos;
      st->error |= err;
      st->max_drift = fmax(st->max_drift, max_drift);
      st->recoveries += recoveries;
      if (sweeps) {
        st->next_rec = next_rec;
        st->rec_every = rec_every;
      }
    }
    __syncthreads();
  }
};

template <class C>
__global__ __launch_bounds__(C::NTH, 1) void window_global_kernel(const ImpDesc* __restrict__ descs,
                                                                  const int32_t* __restrict__ order, int n_items,
                                                                  int* __restrict__ queue, uint8_t* __restrict__ ws) {
  __shared__ GWSmem<C> sm;
  EngineGW<C> e(sm);
  for (;;) {
    if (threadIdx.x == 0) sm.item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(sm.item);  // uniform: the descriptor loads are scalar
    __syncthreads();
    if (it >= n_items) break;
    e.run(descs + order[it], ws);
  }
}

// Update kind of the window kernels in the kernel registry (device-memory G:
// tile-rows per wave 0).
constexpr int kDkWindowGlobal = 3;

template <int LT>
static KernelInfo gwinfo() {
  using C = GWCfg<LT>;
  return KernelInfo{LT, 0, kDkWindowGlobal, C::NTH, sizeof(GWSmem<C>),
                    reinterpret_cast<const void*>(&window_global_kernel<C>)};
}

static const KernelInfo kWindowGlobal[] = {gwinfo<144>(), gwinfo<160>()};

int window_global_kernels(const KernelInfo** list) {
  *list = kWindowGlobal;
  return (int)(sizeof(kWindowGlobal) / sizeof(kWindowGlobal[0]));
}

}  // namespace hfqmc
