// hfqmc_window.h -- gfx950 sweep kernel with window (submatrix) updates.
//
// Same Hirsch-Fye chain as the rank-one register kernel: Metropolis test of
// R = R_up R_dn, R_s = 1 + (1 - G_s[l][l]) d_s, d_s = exp(-2 s lambda s_l) - 1,
// and on acceptance G_s += (d_s/R_s)(G_s[:,l] - e_l) G_s[l,:].  The slices of
// a sweep are visited in windows W of 16 consecutive slices.  A decision in W
// depends only on the diagonal of G, and a flip inside W changes the block
// G[W,W] by a rank-one term built from G[W,W] itself, so every decision of a
// window is taken on the two 16 x 16 blocks G_s[W,W] alone: one wave holds
// them in registers and applies the rank-one updates there (no barrier, no
// global column or row per accept).  The same wave accumulates
// Q_s = prod_j (1 + u_j e_{l_j}^T) restricted to W, u_j the scaled window
// column of accept j.  With S the accepted slices and D_s the diagonal of
// their flip factors, the Hirsch-Fye relation G' = G + (G - 1)(e^{V'-V} - 1)G'
// and G'[W,:] = Q G[W,:] give the update of the whole matrix at the window's
// end as one rank-|S| product
//     G_s += (G_s[:,S] - E_S) P_s G_s[S,:],   P_s = (D_s Q_s)[S,S],
// which every wave applies to its register tiles with v_mfma_f64_16x16x4f64
// (or, for fp32 products, v_mfma_f32_16x16x4f32 products added into the fp64
// tiles).  The from-scratch Dyson solve G = [1 + (1 - G0)(e^V - 1)]^{-1} G0
// uses the same windows, with every slice's potential switched on from V = 0
// (factor exp(V_l) - 1) in place of a Metropolis decision.
//
// Layout: both G_s live in VGPRs as 16 x 16 tiles (lane = 16*(row/4) + col,
// register = row % 4), wave w holding RT consecutive tile-rows of one spin,
// exactly as the rank-one kernel, so the state area and its host readers are
// shared.  Per window the owner of the window's tile-row publishes it in LDS
// (double buffered), every wave stages its tiles of the window's column strip,
// wave 0 scans, publishes P and S, and all waves flush: two barriers per
// window instead of one per accepted flip.
#pragma once
#include "hfqmc_wscan.h"

namespace hfqmc {

template <int LT_, int RT_, int MX_ = 0>
struct WCfg {
  static constexpr int LT = LT_;            // padded slice count (multiple of 16)
  static constexpr int RT = RT_;            // tile-rows per wave
  static constexpr int MX = MX_;            // 1: fp32 products in the window flush
  static constexpr int NT = LT / 16;        // tiles per dimension = windows per sweep
  static constexpr int WPS = NT / RT;       // waves per spin
  static constexpr int NW = 2 * WPS;        // waves per workgroup
  static constexpr int NTH = 64 * NW;
  static constexpr int JW = (LT + 63) / 64;  // 64-slice words of the field masks
  static constexpr int RS = LT + 2;         // row stride of the published tile-row (doubles)
  static constexpr int TS = 17;             // row stride of staged 16 x 16 tiles
  static constexpr int GS = LT + 1;         // row stride of dumped rows (g(tau) estimator)
  static constexpr int DR = LT < 64 ? LT : 64;  // rows per dump block
  static constexpr int MINB = LT <= 64 ? 2 : 1;
  // registers per lane of a wave (VGPRs + AGPRs) when every wave of
  // MINB workgroups is resident, and the flush form: looped where the
  // tiles take half of them or more, or where three or more waves share a
  // SIMD (the unrolled form spills there, and other waves hide the loop's
  // latency)
  static constexpr int BUDGET = 512 / ((NW * MINB + 3) / 4);
  static constexpr bool LOOP = 2 * (RT * NT * 8) >= BUDGET || BUDGET < 256;
  static_assert(LT % 16 == 0 && NT % RT == 0, "bad tile configuration");
  static_assert(NTH >= LT, "measurement needs one thread per tau_k");
  static_assert(DR * GS <= 4 * 16 * RS, "dump block must fit the row buffers");
};

template <class C>
struct WSmem {
  union {
    double rows[2][2][16 * C::RS];  // [buffer][spin]: the window's tile-row of G_s
    double dump[C::DR * C::GS];     // a block of rows of one spin's G
  } u;
  double tb[C::NW][C::RT][16 * C::TS];  // each wave's tiles of the window's column strip
  double pb[2][16 * C::TS];             // P_s = D_s Q_s of the window (window coordinates)
  double diag[2][C::LT];                // diagonals of G_up, G_dn after a measured sweep
  double weiss[2][2 * C::LT];           // G0_s along its diagonals: [LT + i - j] = G0_s[i][j]
  double red[C::NW];
  uint32_t win[4];                      // S mask, |S|, accepted slices (4 bits each, two words)
  int item;
};

template <class C>
struct EngineW {
  static constexpr int LT = C::LT, RT = C::RT, NT = C::NT, JW = C::JW, RS = C::RS, TS = C::TS, GS = C::GS;

  WSmem<C>& sm;
  // thread and wave indices; refresh_ids() re-derives them behind an opaque
  // asm statement at the start of every window and measurement, so the
  // compiler recomputes the addresses built from them there instead of
  // hoisting dozens of them out of the loops into long-lived registers
  int tid, wave, lane, spin, wr, q, c;
  double g[RT][NT][4];                                // this wave's tiles of G_spin
  uint64_t fm[JW];                                    // fields: bit set <=> s = -1 (uniform)
  int buf = 0;                                        // row-buffer parity (uniform)
  int L = 0;
  ImpDesc d;
  // wave-0 counters
  int64_t accepts = 0, nonpos = 0, err = 0;
  double px = 1.0;  // test hook: NaN poisons the blocks the sweep's decisions read

  __device__ __forceinline__ EngineW(WSmem<C>& s)
      : sm(s),
        tid(threadIdx.x),
        wave(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)),
        lane(threadIdx.x & 63),
        spin(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) / C::WPS),
        wr(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) % C::WPS),
        q((threadIdx.x & 63) >> 4),
        c(threadIdx.x & 15) {}

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
    spin = w / C::WPS;
    wr = w % C::WPS;
  }

  template <class F>
  __device__ __forceinline__ void for_tiles(F&& f) {
    static_for<RT>([&](auto rt) __attribute__((always_inline)) {
      static_for<NT>([&](auto tj) __attribute__((always_inline)) {
        static_for<4>([&](auto r) __attribute__((always_inline)) { f(rt, tj, r); });
      });
    });
  }

  __device__ __forceinline__ int field_neg(int m) const {
    const uint64_t w = pick<JW>(fm, m >> 6);
    return (int)((w >> (m & 63)) & 1);
  }

  // ---------------------------------------------------------------- window
  // Owner of tile-row ww of this wave's spin: publish it (all NT tiles).
  __device__ __forceinline__ void publish_rows(int ww, int b) {
    if (ww / RT != wr) return;
    double* dst = sm.u.rows[b][spin] + (4 * q) * RS + c;
    dispatch<RT>(ww % RT, [&](auto rt) __attribute__((always_inline)) {
      static_for<NT>([&](auto tj) __attribute__((always_inline)) {
        static_for<4>([&](auto r) __attribute__((always_inline)) {
          dst[r * RS + 16 * tj] = g[decltype(rt)::value][tj][r];
        });
      });
      __asm__ volatile("" ::: "memory");
    });
  }

  // Every wave: its tiles of column strip ww, row-major 16 x TS each.
  __device__ __forceinline__ void stage_cols(int ww) {
    dispatch<NT>(ww, [&](auto tj) __attribute__((always_inline)) {
      static_for<RT>([&](auto rt) __attribute__((always_inline)) {
        double* dst = sm.tb[wave][rt] + (4 * q) * TS + c;
        static_for<4>([&](auto r) __attribute__((always_inline)) { dst[r * TS] = g[rt][decltype(tj)::value][r]; });
      });
      __asm__ volatile("" ::: "memory");
    });
  }

  // Wave 0: the window's decisions on the diagonal blocks of the published
  // tile-row.
  __device__ __forceinline__ void scan(int ww, int mode, int jf, const uint64_t (&xw)[JW], double* ratio_out,
                                       int b) {
    const int base = 16 * ww;
    const uint32_t fw0 = (uint32_t)(pick<JW>(fm, base >> 6) >> (base & 63)) & 0xFFFFu;
    // factors as values: a conditional over the descriptor's members would
    // select their addresses and keep the whole engine in scratch memory
    const double fa = mode == WM_DYSON ? +d.dset_p : +d.dflip_p;  // sigma s_l = +1
    const double fb = mode == WM_DYSON ? +d.dset_m : +d.dflip_m;  // sigma s_l = -1
    double u = 0.0;
    if (mode == WM_METROPOLIS) u = bperm_d(((base + c) & 63) << 2, u01(pick<JW>(xw, ww >> 2)));
    win_scan<TS>(sm.u.rows[b][0] + (4 * q) * RS + base + c, sm.u.rows[b][1] + (4 * q) * RS + base + c, RS, lane, q,
                 c, base, L, fw0, fa, fb, mode, jf, u, px, ratio_out, sm.pb[0], sm.pb[1], sm.win, accepts, nonpos,
                 err);
  }

  // Every wave: G_s += (G_s[:,S] - E_S) P_s[S,S] G_s[S,:] on its tiles.
  // Per tile-row r: V = P^T (G[r-rows, S] - E)^T (16 x 16, rows = accepted
  // slices in order, columns = the tile's rows permuted so that the update's
  // fp64 accumulator lands in the tile layout), then for every tile column
  // G[r, tj] += V^T G[S, tj]: the accumulator registers of V are the A
  // operands of the update, four accepted slices per instruction.  fp32
  // (mixed kernels, Metropolis windows): fp32 products added into the tiles.
  // Two forms of the same arithmetic (each tile adds the groups of four
  // slices in order, so both give the same bits):
  //  * unrolled: ceil(|S| / 4) is a compile-time count in each of four
  //    branches, every operand load issued before the matrix-core steps;
  //  * looped over the groups (C::LOOP): one code path for every |S|.  Four
  //    branches give each tile four definitions to merge, which the large
  //    shapes with two waves per SIMD cannot hold in registers.
  __device__ __forceinline__ void flush(int ww, int m, uint64_t slist, int b, bool fp32) {
    const bool f32 = C::MX && fp32;
    if constexpr (C::LOOP) {
      flush_loop(ww, m, slist, b, f32);
    } else {
      dispatch<4>((m - 1) >> 2, [&](auto kk) __attribute__((always_inline)) {
        flush_k<decltype(kk)::value + 1>(ww, m, slist, b, f32);
      });
    }
  }

  // x where c holds, else 0.  fp64 kernels: as a product, since with a
  // select the compiler moves the load of x into a branch and every such
  // load then waits for its own round trip (x is finite: an element of G, P
  // or the staged strips).  The kernels with fp32 flush products keep the
  // select form, here and in the g(tau) sums: built with the product form,
  // their chains' drift grew without bound at 48 and 64 slices (the same
  // result on every run), for a reason not found.
  __device__ __forceinline__ static double keep(bool c, double x) {
    if constexpr (C::MX)
      return c ? x : 0.0;
    else
      return x * (c ? 1.0 : 0.0);
  }

  // row of the tile fed as V's column ii: permuted for the fp64 accumulator
  // (rows 4*reg + lane/16), natural for fp32 (rows 4*(lane/16) + reg)
  __device__ __forceinline__ static int v_row(int ii, bool f32) { return f32 ? ii : 4 * (ii & 3) + (ii >> 2); }

  __device__ __forceinline__ void tile_update(double (&t)[4], double a, double rv, bool f32) {
    if (!f32) {
      wd4 acc = {t[0], t[1], t[2], t[3]};
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, rv, acc, 0, 0, 0);
      static_for<4>([&](auto r2) __attribute__((always_inline)) { t[r2] = acc[decltype(r2)::value]; });
    } else {
      wf4 p = {0.f, 0.f, 0.f, 0.f};
      p = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)rv, p, 0, 0, 0);
      static_for<4>([&](auto r2) __attribute__((always_inline)) { t[r2] += (double)p[decltype(r2)::value]; });
    }
  }

  template <int K4>
  __device__ __forceinline__ void flush_k(int ww, int m, uint64_t slist, int b, bool f32) {
    const int ii = lane & 15, qq = lane >> 4;
    const double* pb = sm.pb[spin];
    const double* rows = sm.u.rows[b][spin];
    const int si = (int)(slist >> (4 * ii)) & 15;
    int sk[K4];
    bool kv[K4];
    static_for<K4>([&](auto gi) __attribute__((always_inline)) {
      const int k = 4 * gi + qq;
      kv[gi] = k < m;
      sk[gi] = (int)(slist >> (4 * k)) & 15;
    });
    const int pi = v_row(ii, f32);
    static_for<RT>([&](auto rt) __attribute__((always_inline)) {
      const int r = wr * RT + rt;
      const double* tb = sm.tb[wave][rt];
      double av[K4], bv[K4];
      static_for<K4>([&](auto gi) __attribute__((always_inline)) {
        const double x = pb[sk[gi] * TS + si];
        const double y = tb[pi * TS + sk[gi]] - ((r == ww && pi == sk[gi]) ? 1.0 : 0.0);
        av[gi] = keep(kv[gi] && ii < m, x);
        bv[gi] = keep(kv[gi], y);
      });
      wd4 V = {0.0, 0.0, 0.0, 0.0};
      static_for<K4>([&](auto gi) __attribute__((always_inline)) {
        V = __builtin_amdgcn_mfma_f64_16x16x4f64(av[gi], bv[gi], V, 0, 0, 0);
      });
      static_for<NT>([&](auto tj) __attribute__((always_inline)) {
        double rv[K4];
        static_for<K4>([&](auto gi) __attribute__((always_inline)) {
          rv[gi] = keep(kv[gi], rows[sk[gi] * RS + 16 * tj + ii]);
        });
        static_for<K4>([&](auto gi) __attribute__((always_inline)) {
          tile_update(g[rt][tj], V[decltype(gi)::value], rv[gi], f32);
        });
      });
    });
  }

  __device__ __forceinline__ void flush_loop(int ww, int m, uint64_t slist, int b, bool f32) {
    const int ii = lane & 15, qq = lane >> 4;
    const double* pb = sm.pb[spin];
    const double* rows = sm.u.rows[b][spin];
    const int si = (int)(slist >> (4 * ii)) & 15;
    const int pi = v_row(ii, f32);
    const int K4 = (m + 3) >> 2;
    wd4 V[RT];
    static_for<RT>([&](auto rt) __attribute__((always_inline)) { V[rt] = wd4{0.0, 0.0, 0.0, 0.0}; });
    for (int gi = 0; gi < K4; ++gi) {
      const int k = 4 * gi + qq;
      const bool kv = k < m;
      const int sk = (int)(slist >> (4 * k)) & 15;
      const double av = keep(kv && ii < m, pb[sk * TS + si]);
      static_for<RT>([&](auto rt) __attribute__((always_inline)) {
        const int r = wr * RT + rt;
        const double y = sm.tb[wave][rt][pi * TS + sk] - ((r == ww && pi == sk) ? 1.0 : 0.0);
        V[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, keep(kv, y), V[rt], 0, 0, 0);
      });
    }
    for (int gi = 0; gi < K4; ++gi) {
      const int k = 4 * gi + qq;
      const bool kv = k < m;
      const int sk = (int)(slist >> (4 * k)) & 15;
      double a[RT];  // V[gi] with a uniform gi: selects, not a register-indexed move
      static_for<RT>([&](auto rt) __attribute__((always_inline)) {
        a[rt] = gi == 0 ? V[rt][0] : gi == 1 ? V[rt][1] : gi == 2 ? V[rt][2] : V[rt][3];
      });
      static_for<NT>([&](auto tj) __attribute__((always_inline)) {
        const double rv = keep(kv, rows[sk * RS + 16 * tj + ii]);
        static_for<RT>([&](auto rt) __attribute__((always_inline)) { tile_update(g[rt][tj], a[rt], rv, f32); });
      });
    }
  }

  // One window on every wave.  Returns 1 if a ratio of the window's scan was
  // not a positive number (the same on every thread), else 0.
  __device__ __forceinline__ uint32_t window(int ww, int mode, int jf, const uint64_t (&xw)[JW], double* ratio_out) {
    refresh_ids();
    const int b = buf;
    buf ^= 1;
    publish_rows(ww, b);
    stage_cols(ww);
    __syncthreads();
    if (wave == 0) scan(ww, mode, jf, xw, ratio_out, b);
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
    if (m) flush(ww, m, slist, b, mode == WM_METROPOLIS);
    return (w1 >> 8) & 1u;
  }



  // ---------------------------------------------------------------- measurement
  // Part of S_k = sum_l eps G[(l + k) mod L][l] (eps = -1 where l + k
  // wraps, i.e. for rows i < k) held by dumped rows i in [i0, i0 + n) ∩
  // [0, L) (row i at (i - r0) * GS).  Eight independent partial sums with
  // compile-time indices, so eight loads are in flight at a time.
  __device__ __forceinline__ double diag_part(const double* m, int k, int r0, int i0, int n) const {
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int t0 = 0; t0 < n; t0 += 8) {
      static_for<8>([&](auto u) __attribute__((always_inline)) {
        const int i = i0 + t0 + u;
        const bool ok = t0 + u < n && i < L, wrap = i < k;
        if constexpr (C::MX) {  // the select form (see keep())
          const double x = m[(i - r0) * GS + (wrap ? i - k + L : i - k)];
          a[u] += ok ? (wrap ? -x : x) : 0.0;
        } else {
          // every load at a valid address and unconditional, the element
          // weighted by +-1 or 0: a load feeding a select is moved into a
          // branch, and each then waits for its own round trip
          const int at = ok ? (i - r0) * GS + (wrap ? i - k + L : i - k) : 0;
          a[u] += m[at] * (ok ? (wrap ? -1.0 : 1.0) : 0.0);
        }
      });
    }
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }

  // Write rows [r0, r0 + DR) of this wave's tiles into the dump.
  __device__ __forceinline__ void dump_rows(int r0) {
    static_for<RT>([&](auto rt) __attribute__((always_inline)) {
      const int row0 = (wr * RT + rt) * 16;
      if (row0 >= r0 && row0 < r0 + C::DR) {
        double* dst = sm.u.dump + (row0 - r0 + 4 * q) * GS + c;
        static_for<NT>([&](auto tj) __attribute__((always_inline)) {
          static_for<4>([&](auto r) __attribute__((always_inline)) { dst[r * GS + 16 * tj] = g[rt][tj][r]; });
        });
      }
    });
  }

  // Partial S_k of G_up and G_dn: thread t < NP * L takes k = t % L and the
  // part t / L of every dumped block of rows (NP parts of DR / NP rows);
  // other threads get 0.  The rows buffers are reused for the dump, one spin
  // and DR rows at a time.
  static constexpr int NP = (C::NTH / LT) >= 4 ? 4 : ((C::NTH / LT) >= 2 ? 2 : 1);
  __device__ __forceinline__ void green_sums(double& su_k, double& sd_k) {
    su_k = sd_k = 0.0;
    const int k = tid % L, part = tid / L;
    constexpr int RP = C::DR / NP;  // rows of a block per part
    static_for<2>([&](auto s) __attribute__((always_inline)) {
      for (int r0 = 0; r0 < L; r0 += C::DR) {
        __syncthreads();
        if (spin == s) dump_rows(r0);
        __syncthreads();
        if (part < NP) {
          const double x = diag_part(sm.u.dump, k, r0, r0 + part * RP, RP);
          if (s == 0)
            su_k += x;
          else
            sd_k += x;
        }
      }
    });
    __syncthreads();
  }

  // Diagonal entries of this wave's diagonal tiles into sm.diag.
  __device__ __forceinline__ void write_diag() {
    static_for<RT>([&](auto rt) __attribute__((always_inline)) {
      static_for<NT>([&](auto tj) __attribute__((always_inline)) {
        if (tj == wr * RT + rt && q == (c >> 2)) sm.diag[spin][16 * tj + c] = sel4(d4of(g[rt][tj]), c & 3);
      });
    });
  }

  // G = G0: the antiperiodic Toeplitz matrix of this wave's spin
  // (G0[i][j] = g(tau_{i-j}) for i >= j, -g(tau_{i-j+L}) below), zero in the
  // padding.  Every element is an immediate offset from one address per
  // lane, and the padding is a product with 0, not a branch: a conditional
  // load per element splits the tiles' live ranges and they end in scratch.
  __device__ __forceinline__ void set_weiss() {
    const double* base = sm.weiss[spin] + (LT + 4 * q - c + 16 * (wr * RT) - 16 * (NT - 1));
    for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
      const int i = (wr * RT + rt) * 16 + 4 * q + r, j = tj * 16 + c;
      g[rt][tj][r] = base[16 * (rt - tj + NT - 1) + r] * ((i < L && j < L) ? 1.0 : 0.0);
    });
  }

  // Largest |a - G| over this wave's diagonal tiles, a their earlier copy,
  // reduced over the workgroup.
  __device__ __forceinline__ void copy_diag_tiles(double (&a)[RT][4]) const {
    static_for<RT>([&](auto rt) __attribute__((always_inline)) {
      static_for<NT>([&](auto tj) __attribute__((always_inline)) {
        if (tj == wr * RT + rt)
          static_for<4>([&](auto r) __attribute__((always_inline)) { a[rt][r] = g[rt][tj][r]; });
      });
    });
  }
  __device__ __forceinline__ double diag_tile_drift(const double (&a)[RT][4]) {
    double dr = 0.0;
    static_for<RT>([&](auto rt) __attribute__((always_inline)) {
      static_for<NT>([&](auto tj) __attribute__((always_inline)) {
        if (tj == wr * RT + rt)
          static_for<4>([&](auto r) __attribute__((always_inline)) { dr = fmax(dr, fabs(a[rt][r] - g[rt][tj][r])); });
      });
    });
    dr = wave_max(dr);
    if (lane == 0) sm.red[wave] = dr;
    __syncthreads();
    dr = 0.0;
    for (int w = 0; w < C::NW; ++w) dr = fmax(dr, sm.red[w]);
    __syncthreads();
    return dr;
  }

  __device__ __forceinline__ double* state_ptr(uint8_t* ws) const {
    return reinterpret_cast<double*>(ws + d.off_state) + (size_t)tid * (RT * NT * 4);
  }
  // parked parts of the g(tau) bin sums: 2 NP L doubles in the second
  // 2 LT^2 region of the state area (which these kernels do not otherwise use)
  __device__ __forceinline__ double* gpart_state(uint8_t* ws) const {
    return reinterpret_cast<double*>(ws + d.off_state) + 2 * (size_t)LT * LT;
  }
  __device__ __forceinline__ double* lsum_state(uint8_t* ws) const {
    return reinterpret_cast<double*>(ws + d.off_state) + 4 * (size_t)LT * LT;
  }

  // ---------------------------------------------------------------- item
  // Every window of the item runs from one call site: passes are either a
  // Dyson solve from G0 (first, after every recompute_every sweeps, or the
  // OP_RECOMPUTE item), a Metropolis sweep, or one forced flip (OP_FORCE).
  __device__ __forceinline__ void run(const ImpDesc* desc, uint8_t* ws) {
    d = *desc;
    L = d.L;
    accepts = nonpos = err = 0;
    buf = 0;
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
    for (int i = tid; i < 4 * LT; i += C::NTH) {
      const int s = i / (2 * LT), dd = i % (2 * LT) - LT;  // dd = i - j
      double v = 0.0;
      if (dd >= 0 && dd < L)
        v = wv[s * L + dd];
      else if (dd < 0 && dd > -L)
        v = -wv[s * L + dd + L];
      sm.weiss[s][LT + dd] = v;
    }
    // fields as uniform bit masks
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
    if (flags & F_RESUME) {
      const double* p = state_ptr(ws);
      for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
        g[rt][tj][r] = p[(rt * NT + tj) * 4 + r];
      });
    }
    __syncthreads();

    const bool sweeps = d.op == OP_SWEEPS;
    const int64_t nm = d.n_measure, nb = d.n_bins;
    double su = 0.0, sd = 0.0, sx = 0.0;  // wave 0: per-lane sums of 1-G_up, 1-G_dn and their product
    // thread t < NP L: its part of the running bin sums of g_up(tau_k),
    // g_dn(tau_k), k = t % L; the parts are added in a fixed order when the
    // bin completes, and parked part by part when a launch ends inside a bin,
    // so a chain split over launches sums in exactly the order of one launch
    double gau = 0.0, gad = 0.0;
    int64_t cur_bin = -1;
    bool cont = false;  // this launch starts inside a bin a previous one left open
    if (sweeps) {
      const int64_t m0 = d.sweep_begin - d.n_warmup;
      cont = (flags & F_RESUME) && m0 > 0 && m0 < nm && (m0 * nb) / nm == ((m0 - 1) * nb) / nm;
      if (cont && wave == 0) {
        const double* la = lsum_state(ws);
        su = la[lane];
        sd = la[64 + lane];
        sx = la[128 + lane];
      }
    }
    int64_t proposals = 0;
    double max_drift = 0.0;
    // numeric recovery: a sweep whose scan saw a ratio that was not a
    // positive number is repeated once, from its starting fields and a
    // from-scratch Dyson solve; the repeat failing too leaves the error set
    int attempt = 0, recoveries = 0;
    uint64_t fm0[JW];
    int64_t acc0 = 0, np0 = 0, err0 = 0;

    // pass state
    int64_t w = d.sweep_begin;  // sweep of the next Metropolis pass
    int kf = 0;                 // next forced flip
    int mode = (flags & F_RESUME) ? WM_METROPOLIS : WM_DYSON;
    bool drift = false;         // the Dyson pass measures the drift
    bool measure_after = false; // a measurement of sweep w - 1 follows the Dyson pass
    if (d.op == OP_RECOMPUTE) {
      mode = WM_DYSON;
      drift = (flags & F_RESUME) != 0;
    }
    double dt[RT][4] = {};
    for (;;) {
      // ---- choose the pass
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
        if (drift) copy_diag_tiles(dt);
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
      if (mode == WM_DYSON) set_weiss();  // after the pass's set-up (placed here it does not spill)
      // ---- the pass's windows
      uint32_t bad = 0;
      for (int ww = ww0; ww < ww1; ++ww) bad |= window(ww, mode, jf, xw, rout);
      // ---- after the pass
      bool measure = false;
      if (mode == WM_DYSON) {
        if (drift) {
          const double dr = diag_tile_drift(dt);
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
      refresh_ids();
      const int64_t m = w - 1 - d.n_warmup;
      const int64_t b = (m * nb) / nm;
      double* bp = bins + (size_t)b * NV;
      if (b != cur_bin) {
        gau = gad = 0.0;
        if (cont && tid < NP * L) {
          const double* pk = gpart_state(ws);
          gau = pk[tid];
          gad = pk[NP * L + tid];
        }
        cont = false;
        cur_bin = b;
      }
      write_diag();  // read by wave 0 after the barriers of the g(tau) sums
      {
        double xu, xd;
        green_sums(xu, xd);
        gau += xu / (double)L;
        gad += xd / (double)L;
      }
      if (wave == 0) {
        static_for<JW>([&](auto jj) __attribute__((always_inline)) {
          const int mm = lane + 64 * jj;
          if (mm < L) {
            const double xu = 1.0 - sm.diag[0][mm], xd = 1.0 - sm.diag[1][mm];
            su += xu;
            sd += xd;
            sx += xu * xd;
          }
        });
      }
      if ((m + 1 == nm) || (((m + 1) * nb) / nm != b)) {  // the bin is complete
        // parts 1.. hand their sums to part 0 through the (free) dump area
        const int part = tid / L;
        if (part >= 1 && part < NP) {
          sm.u.dump[(part - 1) * 2 * L + tid % L] = gau;
          sm.u.dump[(part - 1) * 2 * L + L + tid % L] = gad;
        }
        __syncthreads();
        if (tid < L) {
          double xu = gau, xd = gad;
          for (int pp = 1; pp < NP; ++pp) {
            xu += sm.u.dump[(pp - 1) * 2 * L + tid];
            xd += sm.u.dump[(pp - 1) * 2 * L + L + tid];
          }
          bp[tid] = xu;
          bp[L + 1 + tid] = xd;
        }
        __syncthreads();
        cur_bin = -1;
        if (wave == 0) {
          const double nu = wave_sum(su) / (double)L, nd = wave_sum(sd) / (double)L;
          const double dx = wave_sum(sx) / (double)L;
          if (lane == 0) {
            bp[L] = nu;
            bp[2 * L + 1] = nd;
            bp[2 * L + 2] = nu;
            bp[2 * L + 3] = nd;
            bp[2 * L + 4] = dx;
          }
        }
        su = sd = sx = 0.0;
      }
    }
    if (sweeps) {
      // a bin still open when this launch ends: park its running sums
      const int64_t ml = d.sweep_end - 1 - d.n_warmup;
      if (d.sweep_end > d.sweep_begin && ml >= 0 && ml + 1 < nm && ((ml + 1) * nb) / nm == (ml * nb) / nm) {
        if (tid < NP * L) {
          double* pk = gpart_state(ws);
          pk[tid] = gau;
          pk[NP * L + tid] = gad;
        }
        if (wave == 0) {
          double* la = lsum_state(ws);
          la[lane] = su;
          la[64 + lane] = sd;
          la[128 + lane] = sx;
        }
      }
    }

    if (flags & F_SAVE) {
      if (flags & F_SAVE_G) {
        double* p = state_ptr(ws);
        for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
          p[(rt * NT + tj) * 4 + r] = g[rt][tj][r];
        });
      }
      if (wave == 0) {
        static_for<JW>([&](auto jj) __attribute__((always_inline)) {
          const int m = lane + 64 * jj;
          if (m < L) fields[m] = ((fm[jj] >> lane) & 1) ? (int8_t)-1 : (int8_t)1;
        });
      }
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
__global__ __launch_bounds__(C::NTH, C::MINB) void window_kernel(const ImpDesc* __restrict__ descs,
                                                                const int32_t* __restrict__ order, int n_items,
                                                                int* __restrict__ queue, uint8_t* __restrict__ ws) {
  __shared__ WSmem<C> sm;
  EngineW<C> e(sm);
  for (;;) {
    if (threadIdx.x == 0) sm.item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = sm.item;
    __syncthreads();
    if (it >= n_items) break;
    e.run(descs + order[it], ws);
  }
}

// Update kinds of the window kernels in the kernel registry.
constexpr int kDkWindow = 3, kDkWindowMixed = 4;

template <int LT, int RT, int MX = 0>
static KernelInfo winfo() {
  using C = WCfg<LT, RT, MX>;
  return KernelInfo{LT, RT, MX ? kDkWindowMixed : kDkWindow, C::NTH, sizeof(WSmem<C>),
                    reinterpret_cast<const void*>(&window_kernel<C>)};
}

// Window kernels compiled in each translation unit (split for parallel builds).
int window_kernels_fp64(const KernelInfo** list);
int window_kernels_mixed(const KernelInfo** list);

}  // namespace hfqmc
