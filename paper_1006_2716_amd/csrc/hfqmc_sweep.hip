// hfqmc_sweep.hip -- gfx950 kernels of the Hirsch-Fye QMC impurity engine.
//
// One workgroup owns one impurity at a time (persistent, work-queue driven).
// Both spin-resolved L x L Green matrices live in VGPRs as 16 x 16 tiles in
// the accumulator layout of v_mfma_f64_16x16x4f64 (lane = 16*(row/4) + col,
// register = row % 4), spread over NW = 2*NT/RT waves: wave w holds RT
// consecutive tile-rows of one spin.  The method (Hirsch-Fye solver named in
// the paper's "Model and Methods" paragraph, applied to every inequivalent
// site of Eq. (1)/(2) in parallel):
//   ratio   R_s = 1 + (1 - G_s[l][l]) d_s,  d_s = exp(-2 s lambda s_l) - 1
//   accept  u < R_up R_dn  (Metropolis)
//   update  G_s += (d_s/R_s) (G_s[:,l] - e_l) G_s[l,:]   (Sherman-Morrison)
//   Dyson   G = [1 + (1 - G0)(e^V - 1)]^{-1} G0, computed from scratch as L
//           rank-one updates that switch V_l from 0 to s lambda s_l starting
//           at G = G0 (the same identity as a flip, with d = exp(V_l) - 1).
// Decisions need only the diagonal; every wave keeps its own copy of both
// diagonals distributed over its lanes (slice m in lane m % 64), so a
// rejected proposal costs no barrier and no LDS traffic.  An accepted one
// costs one barrier: owners stage column l and row l of G in LDS (double
// buffered), every lane applies the rank-one update to its tiles.
#include <hip/hip_runtime.h>

#include "hfqmc_device.h"

namespace hfqmc {

// ------------------------------------------------------------- configuration
// DK_: 0 = Sherman-Morrison rank-one updates applied to the tiles at once;
// 1 = delayed rank-k updates flushed by v_mfma_f64_16x16x4f64; 2 = delayed
// updates whose product is formed by v_mfma_f32_16x16x4f32 (fp32 operands,
// fp32 product) and added into the fp64 tiles.
template <int LT_, int RT_, int DK_ = 0>
struct Cfg {
  static constexpr int LT = LT_;          // padded slice count (multiple of 16)
  static constexpr int RT = RT_;          // tile-rows per wave
  static constexpr int DK = DK_;
  static constexpr int KP = DK ? 32 : 1;  // panel capacity (largest delay depth)
  static constexpr int NT = LT / 16;      // tiles per matrix dimension
  static constexpr int WPS = NT / RT;     // waves per spin
  static constexpr int NW = 2 * WPS;      // waves per workgroup
  static constexpr int NTH = 64 * NW;     // threads per workgroup
  static constexpr int JW = (LT + 63) / 64;  // slices per lane in slice-distributed vectors
  static constexpr int GS = LT + 1;       // padded LDS row stride of a dumped matrix
  static constexpr int MINB = LT <= 64 ? 2 : 1;  // workgroups per CU the register budget targets
  static constexpr bool DUMP2 = LT <= 64;        // both spins fit the LDS dump area at once
  // rank-one kernels up to 96 slices sum G over a bin's sweeps in LDS and
  // evaluate the g(tau) estimator once per bin (it is linear in G); the sum
  // of both spins takes 2 LT (LT + 1) doubles (149 KiB at LT = 96)
  static constexpr bool ACC = DK == 0 && LT <= 96;
  static_assert(LT % 16 == 0 && NT % RT == 0, "bad tile configuration");
  static_assert(NTH >= 2 * LT, "measurement needs one thread per (spin, tau_k)");
};

template <class C>
struct Stage {
  double col[C::LT];  // column l of G_s
  double row[C::LT];  // row l of G_s
};

template <class C>
struct Smem {
  struct Work {
    Stage<C> stage[2][2];            // [buffer][spin]
    double pa[2][C::KP][C::LT];      // delayed updates: scaled columns a_j of each spin
    double pb[2][C::KP][C::LT];      // delayed updates: rows b_j of each spin
  };
  union {
    Work w;
    double dump[C::ACC ? 2 * C::LT : (C::DUMP2 ? 2 : 1) * C::LT * C::GS];  // G for the g(tau) estimator
  } u;
  double gsum[C::ACC ? 2 * C::LT * C::GS : 1];  // running bin sum of G_up, G_dn (row stride GS)
  double weiss[2][C::LT];  // Weiss samples, zero padded
  double red[C::NW];
  int item;
};

// ------------------------------------------------------------- the engine
template <class C>
struct Engine : SliceState<C::JW> {
  static constexpr int LT = C::LT, RT = C::RT, NT = C::NT, WPS = C::WPS, JW = C::JW, GS = C::GS;
  using Slices = SliceState<C::JW>;
  using Slices::dgu;
  using Slices::dgd;
  using Slices::fpu;
  using Slices::fpd;
  using Slices::sv;

  Smem<C>& sm;
  const int tid, wave, lane, spin, wr, q, c;
  // register state
  double g[RT][NT][4];      // this wave's tiles of G_spin
  int buf;                  // staging double-buffer selector (uniform)
  int kb = 0;               // delayed updates pending in the panels (uniform)
  int kdepth = 1;           // flush when kb reaches this depth
  // item constants (uniform), copied out of memory once per item so that
  // barriers (memory clobbers) do not force reloads in the hot loop
  int L;
  ImpDesc d;

  __device__ __forceinline__ Engine(Smem<C>& s)
      : sm(s),
        tid(threadIdx.x),
        // wave-level values through readfirstlane: the compiler then knows
        // they are uniform and keeps every branch and select on them scalar
        wave(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)),
        lane(threadIdx.x & 63),
        spin(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) / WPS),
        wr(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) % WPS),
        q((threadIdx.x & 63) >> 4),
        c(threadIdx.x & 15),
        buf(0) {}

  __device__ __forceinline__ int row_of(int rt, int r) const { return (wr * RT + rt) * 16 + 4 * q + r; }

  // f(rt, tj, r) over this lane's tile elements, all indices compile-time.
  template <class F>
  __device__ __forceinline__ void for_tiles(F&& f) {
    static_for<RT>([&](auto rt) __attribute__((always_inline)) {
      static_for<NT>([&](auto tj) __attribute__((always_inline)) {
        static_for<4>([&](auto r) __attribute__((always_inline)) { f(rt, tj, r); });
      });
    });
  }
  template <class A, class B, class R>
  __device__ __forceinline__ double gget(A rt, B tj, R r) const {
    return g[decltype(rt)::value][decltype(tj)::value][decltype(r)::value];
  }
  template <class A, class B, class R>
  __device__ __forceinline__ void gset(A rt, B tj, R r, double x) {
    g[decltype(rt)::value][decltype(tj)::value][decltype(r)::value] = x;
  }

  __device__ __forceinline__ void set_field(int jj, int s) { Slices::set_field(jj, s, d.dflip_p, d.dflip_m); }
  __device__ __forceinline__ void flip_field(int l) { Slices::flip_field(l, lane, d.dflip_p, d.dflip_m); }

  // Owners write column l and row l of their spin's G to the staging buffer.
  // Column l lives in tile-column l/16 of the lanes with c == l%16; row l in
  // register l%4 of tile-row l/16 of the lanes with q == (l%16)/4.
  // Uniform branches over compile-time indices pick the values to stage: the
  // lanes with c == l%16 publish column l at this wave's rows, the lanes with
  // q == (l%16)/4 of the wave owning tile-row l/16 publish row l.
  __device__ __forceinline__ void stage(int l) {
    const int tl = l >> 4, cl = l & 15, ql = (l & 15) >> 2, rl = l & 3;
    Stage<C>& mine = sm.u.w.stage[buf][spin];
    if (c == cl) {
      dispatch<NT>(tl, [&](auto tj) __attribute__((always_inline)) {
        static_for<RT>([&](auto rt) __attribute__((always_inline)) {
          static_for<4>([&](auto r) __attribute__((always_inline)) { mine.col[row_of(rt, r)] = gget(rt, tj, r); });
        });
        __asm__ volatile("" ::: "memory");  // keeps the leaves' stores apart (no pointer phi)
      });
    }
    if (q == ql && tl / RT == wr) {
      dispatch<RT * 4>((tl % RT) * 4 + rl, [&](auto k) __attribute__((always_inline)) {
        constexpr int rt = decltype(k)::value / 4, r = decltype(k)::value % 4;
        static_for<NT>([&](auto tj) __attribute__((always_inline)) {
          mine.row[tj * 16 + c] = gget(std::integral_constant<int, rt>{}, tj, std::integral_constant<int, r>{});
        });
        __asm__ volatile("" ::: "memory");
      });
    }
    if constexpr (C::DK == 0) {
      // Rank-one kernels stage G[:,l] - e_l: the diagonal copies equal the
      // tile diagonal bit for bit here, so lane l % 64 of the wave holding
      // row l (the column's stager for that row is in the same wave, its
      // store precedes this one) overwrites entry l with G[l][l] - 1.
      if (tl / RT == wr && lane == (l & 63)) {
        const int jj = l >> 6;
        mine.col[l] = (spin == 0 ? pick<JW>(dgu, jj) : pick<JW>(dgd, jj)) - 1.0;
      }
    }
  }
  __device__ __forceinline__ const double* colp(int s, int l) const { return sm.u.w.stage[buf][s].col; }
  __device__ __forceinline__ const double* rowp(int s, int l) const { return sm.u.w.stage[buf][s].row; }

  // After the barrier: read this lane's a = f (G[:,l] - e_l) and b = G[l,:]
  // values and advance both diagonal copies by the same rank-one term.
  __device__ __forceinline__ void fetch(int l, double fu, double fd, double (&a)[RT][4], double (&b)[NT]) {
    const double* row = rowp(spin, l);
    const double f = spin == 0 ? fu : fd;
    const double* col = colp(spin, l);
    static_for<RT>([&](auto rt) __attribute__((always_inline)) {
      static_for<4>([&](auto r) __attribute__((always_inline)) { a[rt][r] = col[row_of(rt, r)]; });
    });
    static_for<RT>([&](auto rt) __attribute__((always_inline)) {
      static_for<4>([&](auto r) __attribute__((always_inline)) {
        double x = a[rt][r];
        if constexpr (C::DK != 0) {
          if (row_of(rt, r) == l) x -= 1.0;
        }
        a[rt][r] = f * x;
      });
    });
    static_for<NT>([&](auto tj) __attribute__((always_inline)) { b[tj] = row[tj * 16 + c]; });
    const double *cu = colp(0, l), *cd = colp(1, l), *ru = rowp(0, l), *rd = rowp(1, l);
    static_for<JW>([&](auto jj) __attribute__((always_inline)) {
      const int m = lane + 64 * jj;
      if (m < LT) {
        double xu = cu[m], xd = cd[m];
        if constexpr (C::DK != 0) {
          if (m == l) {
            xu -= 1.0;
            xd -= 1.0;
          }
        }
        dgu[jj] = __builtin_fma(fu * xu, ru[m], dgu[jj]);
        dgd[jj] = __builtin_fma(fd * xd, rd[m], dgd[jj]);
      }
    });
    buf ^= 1;
  }

  __device__ __forceinline__ void apply(const double (&a)[RT][4], const double (&b)[NT]) {
    for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
      gset(rt, tj, r, __builtin_fma(a[rt][r], b[tj], gget(rt, tj, r)));
    });
  }

  // G_s += f_s (G_s[:,l] - e_l) G_s[l,:] for both spins (one barrier).
  __device__ __forceinline__ void rank1(int l, double fu, double fd) {
    double a[RT][4], b[NT];
    stage(l);
    __syncthreads();
    fetch(l, fu, fd, a, b);
    apply(a, b);
  }

  // ---- delayed rank-k updates: G = G0 + A B^T with G0 in the tiles ----
  // Column l and row l of the current G are the staged G0 column/row plus the
  // pending terms; the new scaled column a = f (G[:,l] - e_l) and row b =
  // G[l,:] are appended as panel columns, and the diagonal copies advance by
  // a_m b_m.  Work items (spin, column|row, index) are spread over the
  // workgroup.
  __device__ __forceinline__ void delayed_append(int l, double fu, double fd) {
    auto& W = sm.u.w;
    for (int it = tid; it < 4 * LT; it += C::NTH) {
      const int s = it / (2 * LT), v = (it / LT) & 1, i = it % LT;
      if (i >= L) {  // padding rows/columns stay exactly zero
        (v == 0 ? W.pa : W.pb)[s][kb][i] = 0.0;
      } else if (v == 0) {
        double x = W.stage[buf][s].col[i];
        for (int j = 0; j < kb; ++j) x = __builtin_fma(W.pa[s][j][i], W.pb[s][j][l], x);
        if (i == l) x -= 1.0;
        W.pa[s][kb][i] = (s ? fd : fu) * x;
      } else {
        double x = W.stage[buf][s].row[i];
        for (int j = 0; j < kb; ++j) x = __builtin_fma(W.pa[s][j][l], W.pb[s][j][i], x);
        W.pb[s][kb][i] = x;
      }
    }
    __syncthreads();
    static_for<JW>([&](auto jj) __attribute__((always_inline)) {
      const int m = lane + 64 * jj;
      if (m < L) {
        dgu[jj] = __builtin_fma(W.pa[0][kb][m], W.pb[0][kb][m], dgu[jj]);
        dgd[jj] = __builtin_fma(W.pa[1][kb][m], W.pb[1][kb][m], dgd[jj]);
      }
    });
    ++kb;
    buf ^= 1;
  }

  // G0 += A B^T over the kb pending updates, four at a time on the matrix
  // cores.  Lane (i, kk) = (lane % 16, lane / 16) feeds A[row i][kk] and
  // B^T[kk][col i].  The fp64 instruction keeps tile row 4*r + q in lane
  // (q, c) register r, the fp32 one row 4*q + r (the tile layout), so for
  // fp64 the A rows are fed transposed within each 4 x 4 block.
  __device__ __forceinline__ void flush() {
    if constexpr (C::DK != 0) {
      if (kb == 0) return;
      const auto& W = sm.u.w;
      const int ii = lane & 15, kk = lane >> 4;
      const int arow = C::DK == 1 ? 4 * (ii & 3) + (ii >> 2) : ii;
      static_for<RT>([&](auto rt) __attribute__((always_inline)) {
        const int ti = wr * RT + rt;
        static_for<NT>([&](auto tj) __attribute__((always_inline)) {
          if constexpr (C::DK == 1) {
            typedef double d4 __attribute__((ext_vector_type(4)));
            d4 acc = {gget(rt, tj, std::integral_constant<int, 0>{}), gget(rt, tj, std::integral_constant<int, 1>{}),
                      gget(rt, tj, std::integral_constant<int, 2>{}), gget(rt, tj, std::integral_constant<int, 3>{})};
            for (int k0 = 0; k0 < kb; k0 += 4) {
              const int k = k0 + kk;
              const double av = k < kb ? W.pa[spin][k][ti * 16 + arow] : 0.0;
              const double bv = k < kb ? W.pb[spin][k][tj * 16 + ii] : 0.0;
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
            static_for<4>([&](auto r) __attribute__((always_inline)) { gset(rt, tj, r, acc[decltype(r)::value]); });
          } else {
            // fp32 products of four updates at a time, each group added into
            // the fp64 tile (no fp32 sum across groups)
            typedef float f4 __attribute__((ext_vector_type(4)));
            for (int k0 = 0; k0 < kb; k0 += 4) {
              const int k = k0 + kk;
              const float av = k < kb ? (float)W.pa[spin][k][ti * 16 + arow] : 0.f;
              const float bv = k < kb ? (float)W.pb[spin][k][tj * 16 + ii] : 0.f;
              f4 acc = {0.f, 0.f, 0.f, 0.f};
              acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
              static_for<4>([&](auto r) __attribute__((always_inline)) {
                gset(rt, tj, r, gget(rt, tj, r) + (double)acc[decltype(r)::value]);
              });
            }
          }
        });
      });
      __syncthreads();  // the panels are reused after this
      kb = 0;
    }
  }

  __device__ __forceinline__ int scan(int l0, const double (&uv)[JW], double& fu, double& fd, int64_t& nonpos,
                                      int64_t& err) const {
    return Slices::scan(l0, L, lane, uv, fu, fd, nonpos, err);
  }

  // Rebuild the diagonal copies from the tiles (after loading saved state).
  __device__ __forceinline__ void diag_from_tiles() {
    __syncthreads();
    double* dst = sm.u.dump + spin * LT;
    for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
      const int i = row_of(rt, r), j = tj * 16 + c;
      if (i == j) dst[i] = gget(rt, tj, r);
    });
    __syncthreads();
    static_for<JW>([&](auto jj) __attribute__((always_inline)) {
      const int m = lane + 64 * jj;
      dgu[jj] = m < LT ? sm.u.dump[m] : 0.0;
      dgd[jj] = m < LT ? sm.u.dump[LT + m] : 0.0;
    });
    __syncthreads();
  }

  // State area: lane-contiguous, lane (wave, lane) owns RT*NT*4 consecutive
  // doubles, so every element is an immediate offset from one address.
  __device__ __forceinline__ double* state_ptr(uint8_t* ws) const {
    return reinterpret_cast<double*>(ws + d.off_state) + (size_t)tid * (RT * NT * 4);
  }

  // Running bin sums parked in the state area between launches (rank-one
  // kernels up to 64 slices): G sums after the tiles and their snapshot
  // region, lane-contiguous like the tiles; then 3 x 64 per-lane sums.
  __device__ __forceinline__ double* gsum_state(uint8_t* ws) const {
    return reinterpret_cast<double*>(ws + d.off_state) + 2 * (size_t)LT * LT + (size_t)tid * (RT * NT * 4);
  }
  __device__ __forceinline__ double* lsum_state(uint8_t* ws) const {
    return reinterpret_cast<double*>(ws + d.off_state) + 4 * (size_t)LT * LT;
  }
  // This lane's elements of the LDS running sum of its spin's G.
  __device__ __forceinline__ double* gsum_ptr() const {
    return sm.gsum + spin * (LT * GS) + row_of(0, 0) * GS + c;
  }

  __device__ __forceinline__ void save_tiles(uint8_t* ws) {
    double* p = state_ptr(ws);
    for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
      p[(rt * NT + tj) * 4 + r] = gget(rt, tj, r);
    });
  }

  // Test hook: the diagonal copies the ratios read times x (1 leaves them
  // unchanged, NaN poisons them).
  __device__ __forceinline__ void scale_diag(double x) {
    static_for<JW>([&](auto jj) __attribute__((always_inline)) {
      dgu[jj] *= x;
      dgd[jj] *= x;
    });
  }

  __device__ __forceinline__ void load_tiles(uint8_t* ws) {
    const double* p = state_ptr(ws);
    for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
      gset(rt, tj, r, p[(rt * NT + tj) * 4 + r]);
    });
  }

  // Dyson equation from scratch: G = G0, then switch every slice's potential
  // from 0 to s*lambda*s_l by a rank-one update.  Returns max |G_old - G_new|
  // over the diagonal 16 x 16 tiles (uniform) when `drift` is set; the old
  // diagonal tiles are kept in registers meanwhile.
  __device__ __forceinline__ double recompute(uint8_t* ws, bool drift) {
    double dt[RT][4] = {};
    if (drift) {
      static_for<RT>([&](auto rt) __attribute__((always_inline)) {
        static_for<NT>([&](auto tj) __attribute__((always_inline)) {
          if (tj == wr * RT + rt)
            static_for<4>([&](auto r) __attribute__((always_inline)) { dt[rt][r] = gget(rt, tj, r); });
        });
      });
    }
    // G = G0, the antiperiodic matrix of this wave's spin, element by element
    // from the Weiss samples in LDS
    for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
      const int i = row_of(rt, r), j = tj * 16 + c;
      double v = 0.0;
      if (i < L && j < L) v = i >= j ? sm.weiss[spin][i - j] : -sm.weiss[spin][i - j + L];
      gset(rt, tj, r, v);
    });
    {
      const double g0u = sm.weiss[0][0], g0d = sm.weiss[1][0];
      static_for<JW>([&](auto jj) __attribute__((always_inline)) {
        const int m = lane + 64 * jj;
        dgu[jj] = m < L ? g0u : 0.0;
        dgd[jj] = m < L ? g0d : 0.0;
      });
    }
    for (int l = 0; l < L; ++l) {
      const int jj = l >> 6, ln = l & 63;
      const int s = readlane_i(pick<JW>(sv, jj), ln);
      const double du = s > 0 ? d.dset_p : d.dset_m;  // up: V_l = +lambda s_l
      const double dd = s > 0 ? d.dset_m : d.dset_p;  // down: V_l = -lambda s_l
      const double Gu = readlane_d(pick<JW>(dgu, jj), ln), Gd = readlane_d(pick<JW>(dgd, jj), ln);
      const double Ru = __builtin_fma(1.0 - Gu, du, 1.0), Rd = __builtin_fma(1.0 - Gd, dd, 1.0);
      rank1(l, du * recip(Ru), dd * recip(Rd));
    }
    double dr = 0.0;
    if (drift) {
      static_for<RT>([&](auto rt) __attribute__((always_inline)) {
        static_for<NT>([&](auto tj) __attribute__((always_inline)) {
          if (tj == wr * RT + rt)
            static_for<4>([&](auto r) __attribute__((always_inline)) {
              dr = fmax(dr, fabs(dt[rt][r] - gget(rt, tj, r)));
            });
        });
      });
      dr = wave_max(dr);
      if (lane == 0) sm.red[wave] = dr;
      __syncthreads();
      dr = 0.0;
      for (int w = 0; w < C::NW; ++w) dr = fmax(dr, sm.red[w]);
      __syncthreads();
    }
    return dr;
  }

  // g_s(tau_k) sums for this sweep: S_k = sum_l eps G_s[(l+k) mod L][l].
  // The tiles are dumped to LDS (both spins at once when they fit) and
  // thread t = s*L + k adds S_k / L of spin s into gacc.
  __device__ __forceinline__ double diag_sum(const double* m, int k) const {
    // element ((l+k) mod L, l) sits at k*GS + l*(GS+1), minus L*GS once
    // wrapped (l >= L - k).  The same compile-time trip count on every lane,
    // every load unconditional at a valid address and weighted by +-1 or 0:
    // per-lane loop bounds and loads under a condition made each load wait
    // for its own round trip.
    constexpr int S = GS + 1;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    // opaque: the addresses are not loop-invariant to the compiler, which
    // would otherwise keep all of them (and their weights) in registers
    // across the whole sweep loop
    __asm__ volatile("" : "+v"(k));
    const int nw = L - k;
    const double* p0 = m + k * GS;
#pragma unroll 2
    for (int l0 = 0; l0 < LT; l0 += 4) {
      static_for<4>([&](auto u) __attribute__((always_inline)) {
        const int l = l0 + u;
        const bool ok = l < L, wrap = l >= nw;
        const int at = ok ? (wrap ? l * S - L * GS : l * S) : -k * GS;
        a[u] += p0[at] * (ok ? (wrap ? -1.0 : 1.0) : 0.0);
      });
    }
    return (a[0] + a[1]) + (a[2] + a[3]);
  }

  __device__ __forceinline__ void dump_tiles(double* m) {
    double* dst = m + row_of(0, 0) * GS + c;
    for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
      dst[(rt * 16 + r) * GS + tj * 16] = gget(rt, tj, r);
    });
  }

  __device__ __forceinline__ void measure_green(double& gacc) {
    __syncthreads();  // the dump area aliases the staging buffers
    if constexpr (C::DUMP2) {
      dump_tiles(sm.u.dump + spin * (LT * GS));
      __syncthreads();
      if (tid < 2 * L) {
        const int s = tid >= L, k = tid - s * L;
        gacc += diag_sum(sm.u.dump + s * (LT * GS), k) / (double)L;
      }
    } else {
      static_for<2>([&](auto s) __attribute__((always_inline)) {
        if (spin == s) dump_tiles(sm.u.dump);
        __syncthreads();
        if (tid >= s * L && tid < (s + 1) * L) gacc += diag_sum(sm.u.dump, tid - s * L) / (double)L;
        if (s == 0) __syncthreads();
      });
    }
    __syncthreads();  // the next staging write reuses the dump area
  }

  __device__ __forceinline__ void run(const ImpDesc* desc, uint8_t* ws) {
    d = *desc;
    L = d.L;
    kdepth = d.delay < 1 ? 1 : (d.delay > C::KP ? C::KP : d.delay);
    kb = 0;
    const int flags = d.flags;
    const int NV = n_values(L);
    double* bins = reinterpret_cast<double*>(ws + d.off_bins);
    ImpStatus* st = reinterpret_cast<ImpStatus*>(ws + d.off_status);
    int8_t* fields = reinterpret_cast<int8_t*>(ws + d.off_fields);
    const double* wv = reinterpret_cast<const double*>(ws + d.off_weiss);

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
    // fields
    if (flags & (F_FIELDS_GIVEN | F_RESUME | F_KEEP_FIELDS)) {
      const int8_t* fin = (flags & F_FIELDS_GIVEN) ? reinterpret_cast<const int8_t*>(ws + d.off_init) : fields;
      static_for<JW>([&](auto jj) __attribute__((always_inline)) {
        const int m = lane + 64 * jj;
        set_field(jj, m < L ? (fin[m] < 0 ? -1 : 1) : 1);
      });
    } else {
      const U64x4 x = philox4x64_10((uint64_t)lane, 0, kPurposeInit, (uint64_t)d.chain, d.seed, d.site);
      static_for<JW>([&](auto jj) __attribute__((always_inline)) { set_field(jj, (x.v[jj] >> 63) ? -1 : 1); });
    }
    __syncthreads();
    if (flags & F_RESUME) {
      load_tiles(ws);
      diag_from_tiles();
    } else {
      recompute(ws, false);
    }

    int64_t proposals = 0, accepts = 0, nonpos = 0;
    int64_t err = 0;
    double max_drift = 0.0;
    int recoveries = 0;

    if (d.op == OP_SWEEPS) {
      // Running bin sums.  They are loaded when a bin is entered and stored
      // (not added) when it is left or the launch ends, so a chain split
      // over several launches sums in exactly the order of one launch.
      double gacc = 0.0;  // thread t < 2L: running bin sum of g_s(tau_k), s = t / L, k = t % L
      double nacc_u = 0.0, nacc_d = 0.0, dacc = 0.0;
      int64_t cur_bin = -1;
      const int64_t nm = d.n_measure, nb = d.n_bins;
      // ACC kernels: lane sums over the bin's sweeps of 1 - G_up[m][m],
      // 1 - G_dn[m][m] and their product (slices m = lane + 64 jj), and the LDS sum
      // of G; a bin that a previous launch left open continues from the
      // sums it parked, so a split chain adds in the order of one launch
      double su = 0.0, sd = 0.0, sx = 0.0;
      if constexpr (C::ACC) {
        const int64_t m0 = d.sweep_begin - d.n_warmup;
        const bool cont = (flags & F_RESUME) && m0 > 0 && m0 < nm && (m0 * nb) / nm == ((m0 - 1) * nb) / nm;
        double* gp = gsum_ptr();
        if (cont) {
          const double* src = gsum_state(ws);
          for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
            gp[(rt * 16 + r) * GS + tj * 16] = src[(rt * NT + tj) * 4 + r];
          });
          const double* la = lsum_state(ws);
          su = la[lane];
          sd = la[64 + lane];
          sx = la[128 + lane];
        } else {
          for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
            gp[(rt * 16 + r) * GS + tj * 16] = 0.0;
          });
        }
      }
      // numeric recovery: a sweep whose scan saw a ratio that was not a
      // positive number is repeated once, from its starting fields and a
      // from-scratch Dyson solve; the repeat failing too leaves the error set
      int attempt = 0;
      for (int64_t w = d.sweep_begin; w < d.sweep_end; ++w) {
        uint64_t fl[JW];  // slices flipped in this sweep (uniform)
        static_for<JW>([&](auto jj) __attribute__((always_inline)) { fl[jj] = 0; });
        const int64_t pr0 = proposals, acc0 = accepts, np0 = nonpos, err0 = err;
        scale_diag((attempt ? +d.poison[1] : +d.poison[0]) == w + 1 ? __builtin_nan("") : 1.0);
        double uv[JW];
        {
          const U64x4 x = philox4x64_10((uint64_t)lane, (uint64_t)(w + d.rng_offset), kPurposeSweep,
                                        (uint64_t)d.chain, d.seed, d.site);
          static_for<JW>([&](auto jj) __attribute__((always_inline)) { uv[jj] = u01(x.v[jj]); });
        }
        double fu, fd;
        int l = scan(0, uv, fu, fd, nonpos, err);
        int l0 = 0;
        while (l < L) {
          if constexpr (C::DK == 0) {
            // accepted flip of slice l: stage, then the rank-one update; the
            // scan for the next accepted slice only needs the new diagonals,
            // so it is issued before the tile FMAs to overlap their latency
            double a[RT][4], b[NT];
            stage(l);
            __syncthreads();
            fetch(l, fu, fd, a, b);
            flip_field(l);
            mark_flip(fl, l);
            proposals += l - l0 + 1;
            ++accepts;
            l0 = l + 1;
            l = scan(l0, uv, fu, fd, nonpos, err);
            apply(a, b);
          } else {
            stage(l);
            __syncthreads();
            delayed_append(l, fu, fd);
            if (kb >= kdepth) flush();
            flip_field(l);
            mark_flip(fl, l);
            proposals += l - l0 + 1;
            ++accepts;
            l0 = l + 1;
            l = scan(l0, uv, fu, fd, nonpos, err);
          }
        }
        flush();
        proposals += L - l0;
        const bool retry = nonpos != np0 && attempt == 0;
        attempt = retry;
        if (retry) {  // back to the sweep's starting state
          static_for<JW>([&](auto jj) __attribute__((always_inline)) {
            if ((fl[jj] >> lane) & 1) set_field(jj, -sv[jj]);
          });
          proposals = pr0;
          accepts = acc0;
          nonpos = np0;
          err = err0;
          ++recoveries;
        }
        if (retry || w == next_rec) {
          const double dr = recompute(ws, !retry);
          if (!retry) {
            max_drift = fmax(max_drift, dr);
            if (d.drift_limit > 0.0 && !(dr <= d.drift_limit)) {
              if (rec_every > 1)
                rec_every >>= 1;
              else
                err = 1;
            }
            next_rec += rec_every;
          }
        }
        if (retry) {
          --w;
          continue;
        }
        if (C::ACC && w >= d.n_warmup) {
          const int64_t m = w - d.n_warmup;
          const int64_t b = (m * nb) / nm;
          double* gp = gsum_ptr();
          for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
            gp[(rt * 16 + r) * GS + tj * 16] += gget(rt, tj, r);
          });
          static_for<JW>([&](auto jj) __attribute__((always_inline)) {
            if (lane + 64 * jj < L) {
              su += 1.0 - dgu[jj];
              sd += 1.0 - dgd[jj];
              sx += (1.0 - dgu[jj]) * (1.0 - dgd[jj]);
            }
          });
          if ((m + 1 == nm) || (((m + 1) * nb) / nm != b)) {  // the bin is complete: evaluate it
            __syncthreads();
            double* bp = bins + (size_t)b * NV;
            if (tid < 2 * L) {
              const int sp = tid >= L, k = tid - sp * L;
              bp[tid + (tid >= L)] = diag_sum(sm.gsum + sp * (LT * GS), k) / (double)L;
            }
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
            __syncthreads();
            for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
              gp[(rt * 16 + r) * GS + tj * 16] = 0.0;
            });
            su = sd = sx = 0.0;
          }
        } else if (w >= d.n_warmup) {
          const int64_t m = w - d.n_warmup;
          const int64_t b = (m * nb) / nm;
          double* bp = bins + (size_t)b * NV;
          if (b != cur_bin) {
            gacc = tid < 2 * L ? bp[tid + (tid >= L)] : 0.0;
            nacc_u = bp[2 * L + 2];
            nacc_d = bp[2 * L + 3];
            dacc = bp[2 * L + 4];
            cur_bin = b;
          }
          // density and double occupancy from the diagonals
          double xu = 0.0, xd = 0.0, xx = 0.0;
          static_for<JW>([&](auto jj) __attribute__((always_inline)) {
            const int mm = lane + 64 * jj;
            if (mm < L) {
              xu += 1.0 - dgu[jj];
              xd += 1.0 - dgd[jj];
              xx += (1.0 - dgu[jj]) * (1.0 - dgd[jj]);
            }
          });
          nacc_u += wave_sum(xu) / (double)L;
          nacc_d += wave_sum(xd) / (double)L;
          dacc += wave_sum(xx) / (double)L;
          if constexpr (!C::ACC) measure_green(gacc);
          const bool last = (m + 1 == nm) || (((m + 1) * nb) / nm != b) || (w + 1 == d.sweep_end);
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
      }
      if constexpr (C::ACC) {
        // a bin still open when this launch ends: park its running sums
        const int64_t ml = d.sweep_end - 1 - d.n_warmup;
        if (d.sweep_end > d.sweep_begin && ml >= 0 && ml + 1 < nm && ((ml + 1) * nb) / nm == (ml * nb) / nm) {
          const double* gp = gsum_ptr();
          double* dst = gsum_state(ws);
          for_tiles([&](auto rt, auto tj, auto r) __attribute__((always_inline)) {
            dst[(rt * NT + tj) * 4 + r] = gp[(rt * 16 + r) * GS + tj * 16];
          });
          if (wave == 0) {
            double* la = lsum_state(ws);
            la[lane] = su;
            la[64 + lane] = sd;
            la[128 + lane] = sx;
          }
        }
      }
    } else if (d.op == OP_FORCE) {
      const int32_t* slices = reinterpret_cast<const int32_t*>(ws + d.off_force);
      double* ratios = reinterpret_cast<double*>(ws + d.off_force + 4 * ((d.n_force + 1) & ~1));
      for (int k = 0; k < d.n_force; ++k) {
        const int l = slices[k];
        const int jj = l >> 6, ln = l & 63;
        const double Gu = readlane_d(pick<JW>(dgu, jj), ln), Gd = readlane_d(pick<JW>(dgd, jj), ln);
        const double du = readlane_d(pick<JW>(fpu, jj), ln), dd = readlane_d(pick<JW>(fpd, jj), ln);
        const double Ru = __builtin_fma(1.0 - Gu, du, 1.0), Rd = __builtin_fma(1.0 - Gd, dd, 1.0);
        if (tid == 0) ratios[k] = Ru * Rd;
        rank1(l, du * recip(Ru), dd * recip(Rd));
        flip_field(l);
      }
    } else if (d.op == OP_RECOMPUTE) {
      max_drift = recompute(ws, true);
    }

    if (flags & F_SAVE) {
      if (flags & F_SAVE_G) save_tiles(ws);
      if (wave == 0) {
        static_for<JW>([&](auto jj) __attribute__((always_inline)) {
          const int m = lane + 64 * jj;
          if (m < L) fields[m] = (int8_t)sv[jj];
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
      if (d.op == OP_SWEEPS) {
        st->next_rec = next_rec;
        st->rec_every = rec_every;
      }
    }
    __syncthreads();
  }
};

template <class C>
__global__ __launch_bounds__(C::NTH, C::MINB) void sweep_kernel(const ImpDesc* __restrict__ descs, const int32_t* __restrict__ order,
                                                       int n_items, int* __restrict__ queue, uint8_t* __restrict__ ws) {
  __shared__ Smem<C> sm;
  Engine<C> e(sm);
  for (;;) {
    if (threadIdx.x == 0) sm.item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = sm.item;
    __syncthreads();
    if (it >= n_items) break;
    e.run(descs + order[it], ws);
  }
}

__global__ void zero_kernel(uint64_t* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// ------------------------------------------------------------- host dispatch
template <int LT, int RT, int DK = 0>
static KernelInfo info() {
  using C = Cfg<LT, RT, DK>;
  return KernelInfo{LT, RT, DK, C::NTH, sizeof(Smem<C>), reinterpret_cast<const void*>(&sweep_kernel<C>)};
}

static const KernelInfo kKernels[] = {
    info<16, 1>(), info<32, 1>(), info<32, 2>(), info<48, 1>(), info<48, 3>(), info<64, 1>(), info<64, 2>(),
    info<64, 4>(), info<80, 1>(), info<96, 1>(), info<96, 2>(), info<96, 3>(), info<112, 1>(), info<128, 1>(),
    info<128, 2>(),
    // delayed rank-k updates, fp64 and mixed-precision flushes
    info<32, 1, 1>(), info<48, 1, 1>(), info<64, 2, 1>(), info<80, 1, 1>(), info<96, 1, 1>(), info<128, 1, 1>(),
    info<32, 1, 2>(), info<48, 1, 2>(), info<64, 2, 2>(), info<80, 1, 2>(), info<96, 1, 2>(), info<128, 1, 2>(),
};

// Every compiled kernel: the rank-one and delayed register kernels of this
// unit, the window kernels and the global-memory kernels.
template <class F>
static const KernelInfo* each_kernel(F&& f) {
  for (const auto& k : kKernels)
    if (f(k)) return &k;
  const KernelInfo* lists[3] = {nullptr, nullptr, nullptr};
  const int counts[3] = {window_kernels(&lists[0]), global_kernels(&lists[1]), window_global_kernels(&lists[2])};
  for (int l = 0; l < 3; ++l)
    for (int i = 0; i < counts[l]; ++i)
      if (f(lists[l][i])) return &lists[l][i];
  return nullptr;
}

const KernelInfo* find_kernel(int LT, int RT, int DK) {
  return each_kernel([&](const KernelInfo& k) { return k.LT == LT && k.RT == RT && k.DK == DK; });
}

// Tile-rows-per-wave variants compiled for (LT, DK), 0 standing for the
// global-memory kernel; returns their count.
int kernel_variants(int LT, int DK, int* rt_out, int max) {
  int n = 0;
  each_kernel([&](const KernelInfo& k) {
    if (k.LT == LT && k.DK == DK) {
      if (n < max) rt_out[n] = k.RT;
      ++n;
    }
    return false;
  });
  return n;
}

int kernel_threads(const KernelInfo* k) { return k->threads; }
size_t kernel_lds(const KernelInfo* k) { return k->lds; }

hipError_t kernel_occupancy(const KernelInfo* k, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k->fn, k->threads, 0);
}

hipError_t launch_sweep(const KernelInfo* k, int grid, hipStream_t st, const ImpDesc* descs, const int32_t* order,
                        int n_items, int* queue, uint8_t* ws) {
  void* args[] = {(void*)&descs, (void*)&order, (void*)&n_items, (void*)&queue, (void*)&ws};
  return hipLaunchKernel(k->fn, dim3(grid), dim3(k->threads), args, 0, st);
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 8;
  if (n == 0) return hipSuccess;
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(256), 0, st, reinterpret_cast<uint64_t*>(p), n);
  return hipGetLastError();
}

}  // namespace hfqmc
