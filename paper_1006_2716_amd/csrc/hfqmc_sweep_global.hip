// hfqmc_sweep_global.hip -- gfx950 sweep kernel for imaginary-time grids
// whose two L x L Green matrices do not fit the register file (both spins at
// L = 160 take 400 KiB of the 512 KiB a CU has).
//
// Same Hirsch-Fye chain as the register-tile kernel (ratio, Metropolis test,
// Dyson by forced updates, estimators), but G_s lives in HBM -- row-major,
// padded to LT, in the impurity's state area, where it stays resident in L2
// while its workgroup runs -- and every accepted flip is a delayed update:
//   current column c = G0[:,l] + A B[l,:]^T,  row r = G0[l,:] + A[l,:] B^T
//   append   a = (d_s/R_s)(c - e_l)  as a new column of A,  b = r of B
//   flush    G0 += A B^T on the matrix cores (v_mfma_f64_16x16x4f64) once k
//            updates are pending, at the end of every sweep, and before any
//            measurement or Dyson recompute.
// The panels A, B (k <= 16 per spin) are in LDS; per accept the workgroup
// reads one column and one row of G0 per spin from L2, and G0 streams
// through the CU once per k accepts.
#include "hfqmc_device.h"

namespace hfqmc {

template <int LT_>
struct GCfg {
  static constexpr int LT = LT_;
  static constexpr int NT = LT / 16;
  static constexpr int NW = 8;               // waves per workgroup
  static constexpr int NTH = 64 * NW;
  static constexpr int JW = (LT + 63) / 64;  // slices per lane in slice-distributed vectors
  static constexpr int KP = 16;              // panel capacity (largest delay depth)
  static constexpr int RB = 4 * KP;          // rows of G per measurement chunk (aliases the panels)
  static_assert(LT % 16 == 0 && NTH >= 2 * LT, "bad configuration");
};

template <class C>
struct GSmem {
  union {
    struct {
      double pa[2][C::KP][C::LT];  // scaled columns a_j of each spin
      double pb[2][C::KP][C::LT];  // rows b_j of each spin
    } p;
    double rows[C::RB * C::LT];    // a block of rows of G_s for the g(tau) estimator
  } u;
  double weiss[2][C::LT];
  double red[C::NW];
  int item;
};

template <class C>
struct EngineG : SliceState<C::JW> {
  static constexpr int LT = C::LT, NT = C::NT, JW = C::JW, KP = C::KP;
  typedef double d4 __attribute__((ext_vector_type(4)));
  using Slices = SliceState<C::JW>;
  using Slices::dgu;
  using Slices::dgd;
  using Slices::fpu;
  using Slices::fpd;
  using Slices::sv;

  GSmem<C>& sm;
  const int tid, wave, lane;
  int kb = 0;               // pending delayed updates (uniform)
  int kdepth = KP;          // flush depth
  int L = 0;
  ImpDesc d;
  double* gm = nullptr;     // G_up, G_dn (LT x LT each), then the drift snapshot of both

  __device__ __forceinline__ EngineG(GSmem<C>& s)
      : sm(s), tid(threadIdx.x), wave(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)), lane(threadIdx.x & 63) {}

  __device__ __forceinline__ void set_field(int jj, int s) { Slices::set_field(jj, s, d.dflip_p, d.dflip_m); }
  __device__ __forceinline__ void flip_field(int l) { Slices::flip_field(l, lane, d.dflip_p, d.dflip_m); }

  // Stores of every wave to G visible to the loads of every wave: the
  // workgroup-scope release/acquire of the barrier suffices (the waves share
  // the CU's caches); a device-scope fence would write back and invalidate
  // the whole L2 each time.
  __device__ __forceinline__ void publish() { __syncthreads(); }

  __device__ __forceinline__ int scan(int l0, const double (&uv)[JW], double& fu, double& fd, int64_t& nonpos,
                                      int64_t& err) const {
    return Slices::scan(l0, L, lane, uv, fu, fd, nonpos, err);
  }

  // Append the update of slice l with factors f_s = d_s / R_s: column and row
  // of the current G from G0 in memory plus the pending panel terms.
  __device__ __forceinline__ void append(int l, double fu, double fd) {
    auto& P = sm.u.p;
    // work items (spin, column|row, index) tid, tid + NTH, ...: every G0 load
    // of a thread is issued before the first is used (above 128 slices a
    // quarter of the threads take two items; one memory round trip, not two)
    constexpr int NI = (4 * LT + C::NTH - 1) / C::NTH;
    double g0[NI];
    static_for<NI>([&](auto k) __attribute__((always_inline)) {
      const int it = tid + k * C::NTH;
      const int s = it / (2 * LT), v = (it / LT) & 1, i = it % LT;
      const double* Gs = gm + (size_t)s * LT * LT;
      g0[k] = (it < 4 * LT && i < L) ? (v == 0 ? Gs[(size_t)i * LT + l] : Gs[(size_t)l * LT + i]) : 0.0;
    });
    static_for<NI>([&](auto k) __attribute__((always_inline)) {
      const int it = tid + k * C::NTH;
      if (it < 4 * LT) {
        const int s = it / (2 * LT), v = (it / LT) & 1, i = it % LT;
        if (i >= L) {  // padding rows/columns stay exactly zero
          (v == 0 ? P.pa : P.pb)[s][kb][i] = 0.0;
        } else if (v == 0) {
          double x = g0[k];
#pragma unroll
          for (int j = 0; j < KP; ++j)  // unrolled: all panel reads issue at once
            if (j < kb) x = __builtin_fma(P.pa[s][j][i], P.pb[s][j][l], x);
          if (i == l) x -= 1.0;
          P.pa[s][kb][i] = (s ? fd : fu) * x;
        } else {
          double x = g0[k];
#pragma unroll
          for (int j = 0; j < KP; ++j)
            if (j < kb) x = __builtin_fma(P.pa[s][j][l], P.pb[s][j][i], x);
          P.pb[s][kb][i] = x;
        }
      }
    });
    __syncthreads();
    static_for<JW>([&](auto jj) __attribute__((always_inline)) {
      const int m = lane + 64 * jj;
      if (m < L) {
        dgu[jj] = __builtin_fma(P.pa[0][kb][m], P.pb[0][kb][m], dgu[jj]);
        dgd[jj] = __builtin_fma(P.pa[1][kb][m], P.pb[1][kb][m], dgd[jj]);
      }
    });
    ++kb;
  }

  // G0 += A B^T, four pending updates per matrix-core step.  Wave w takes
  // tiles w, w + NW, ... in groups of U; the loads of the next group are in
  // flight while the matrix cores work on the current one.  Lane (q, c) =
  // (lane / 16, lane % 16) holds tile row 4 r + q, column c in accumulator
  // register r, and feeds A[row c][k0 + q], B[k0 + q][col c].
  __device__ __forceinline__ double* tile_ptr(int t, int q, int c) const {
    const int s = t / (NT * NT), ti = (t / NT) % NT, tj = t % NT;
    return gm + (size_t)s * LT * LT + (size_t)(16 * ti + q) * LT + 16 * tj + c;
  }

  __device__ __forceinline__ void flush() {
    if (kb == 0) return;
    const auto& P = sm.u.p;
    const int q = lane >> 4, c = lane & 15;
    constexpr int NTILE = 2 * NT * NT, U = 4, STEP = C::NW * U;
    d4 cur[U], nxt[U];
    auto load = [&](int t0, d4 (&acc)[U]) __attribute__((always_inline)) {
      static_for<U>([&](auto u) __attribute__((always_inline)) {
        const int t = t0 + u * C::NW;
        if (t < NTILE) {
          const double* g = tile_ptr(t, q, c);
          acc[u] = d4{g[0], g[4 * LT], g[8 * LT], g[12 * LT]};
        }
      });
    };
    if (wave < NTILE) load(wave, cur);
    for (int t0 = wave; t0 < NTILE; t0 += STEP) {
      if (t0 + STEP < NTILE) load(t0 + STEP, nxt);
#pragma unroll
      for (int k0 = 0; k0 < KP; k0 += 4) {  // unrolled over the panel capacity: fragment reads issue together
        if (k0 >= kb) break;
        const int k = k0 + q;
        static_for<U>([&](auto u) __attribute__((always_inline)) {
          const int t = t0 + u * C::NW;
          const int tt = t < NTILE ? t : t0;
          const int s = tt / (NT * NT), ti = (tt / NT) % NT, tj = tt % NT;
          const double av = k < kb ? P.pa[s][k][16 * ti + c] : 0.0;
          const double bv = k < kb ? P.pb[s][k][16 * tj + c] : 0.0;
          cur[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, cur[u], 0, 0, 0);
        });
      }
      static_for<U>([&](auto u) __attribute__((always_inline)) {
        const int t = t0 + u * C::NW;
        if (t < NTILE) {
          double* g = tile_ptr(t, q, c);
          g[0] = cur[u][0];
          g[4 * LT] = cur[u][1];
          g[8 * LT] = cur[u][2];
          g[12 * LT] = cur[u][3];
        }
        cur[u] = nxt[u];
      });
    }
    publish();  // also frees the panels
    kb = 0;
  }

  // Test hook: the diagonal copies the ratios read times x (1 leaves them
  // unchanged, NaN poisons them).
  __device__ __forceinline__ void scale_diag(double x) {
    static_for<JW>([&](auto jj) __attribute__((always_inline)) {
      dgu[jj] *= x;
      dgd[jj] *= x;
    });
  }

  __device__ __forceinline__ void diag_from_memory() {
    static_for<JW>([&](auto jj) __attribute__((always_inline)) {
      const int m = lane + 64 * jj;
      dgu[jj] = m < L ? gm[(size_t)m * LT + m] : 0.0;
      dgd[jj] = m < L ? gm[(size_t)LT * LT + (size_t)m * LT + m] : 0.0;
    });
  }

  // Dyson equation from scratch: G = G0, then switch every slice's potential
  // from 0 to s*lambda*s_l by forced delayed updates.  Returns max |G_old -
  // G_new| (uniform) when `drift` is set (G_old parked after both matrices).
  __device__ __forceinline__ double recompute(bool drift) {
    double* old = gm + 2 * (size_t)LT * LT;
    for (int idx = tid; idx < 2 * LT * LT; idx += C::NTH) {
      const int s = idx / (LT * LT), i = (idx / LT) % LT, j = idx % LT;
      double v = 0.0;
      if (i < L && j < L) v = i >= j ? sm.weiss[s][i - j] : -sm.weiss[s][i - j + L];
      if (drift) old[idx] = gm[idx];
      gm[idx] = v;
    }
    publish();
    {
      const double g0u = sm.weiss[0][0], g0d = sm.weiss[1][0];
      static_for<JW>([&](auto jj) __attribute__((always_inline)) {
        const int m = lane + 64 * jj;
        dgu[jj] = m < L ? g0u : 0.0;
        dgd[jj] = m < L ? g0d : 0.0;
      });
    }
    kb = 0;
    for (int l = 0; l < L; ++l) {
      const int jj = l >> 6, ln = l & 63;
      const int s = readlane_i(pick<JW>(sv, jj), ln);
      const double du = s > 0 ? d.dset_p : d.dset_m;  // up: V_l = +lambda s_l
      const double dd = s > 0 ? d.dset_m : d.dset_p;  // down: V_l = -lambda s_l
      const double Gu = readlane_d(pick<JW>(dgu, jj), ln), Gd = readlane_d(pick<JW>(dgd, jj), ln);
      const double Ru = __builtin_fma(1.0 - Gu, du, 1.0), Rd = __builtin_fma(1.0 - Gd, dd, 1.0);
      append(l, du * recip(Ru), dd * recip(Rd));
      if (kb >= kdepth) flush();
    }
    flush();
    double dr = 0.0;
    if (drift) {
      for (int idx = tid; idx < 2 * LT * LT; idx += C::NTH) dr = fmax(dr, fabs(old[idx] - gm[idx]));
      dr = wave_max(dr);
      if (lane == 0) sm.red[wave] = dr;
      __syncthreads();
      dr = 0.0;
      for (int w = 0; w < C::NW; ++w) dr = fmax(dr, sm.red[w]);
      __syncthreads();
    }
    return dr;
  }

  // g_s(tau_k) sums S_k = sum_l eps G_s[(l+k) mod L][l] of the flushed G,
  // staged through LDS in blocks of rows; thread t = s*L + k adds S_k / L.
  __device__ __forceinline__ void measure_green(double& gacc) {
    const int sme = tid >= L, k = tid - sme * L;
    double S = 0.0;
    for (int s = 0; s < 2; ++s) {
      const double* Gs = gm + (size_t)s * LT * LT;
      for (int r0 = 0; r0 < L; r0 += C::RB) {
        const int r1 = r0 + C::RB < L ? r0 + C::RB : L;
        __syncthreads();
        {  // every load of a thread in flight before its first LDS store
          constexpr int NR = (C::RB * LT + C::NTH - 1) / C::NTH;
          const int n = (r1 - r0) * LT;
          const double* src = Gs + (size_t)r0 * LT;
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
        __syncthreads();
        if (tid < 2 * L && sme == s) {
          const double* R = sm.u.rows;
          int lo = r0 - k > 0 ? r0 - k : 0, hi = (L - k) < (r1 - k) ? (L - k) : (r1 - k);
          for (int l = lo; l < hi; ++l) S += R[(l + k - r0) * LT + l];           // row l + k
          lo = (L - k) > (r0 - k + L) ? (L - k) : (r0 - k + L);
          hi = L < (r1 - k + L) ? L : (r1 - k + L);
          for (int l = lo; l < hi; ++l) S -= R[(l + k - L - r0) * LT + l];       // row l + k - L
        }
      }
    }
    __syncthreads();  // the panels reuse the row buffer
    if (tid < 2 * L) gacc += S / (double)L;
  }

  __device__ __forceinline__ void run(const ImpDesc* desc, uint8_t* ws) {
    d = *desc;
    L = d.L;
    kdepth = d.delay < 1 ? KP : (d.delay > KP ? KP : d.delay);
    kb = 0;
    gm = reinterpret_cast<double*>(ws + d.off_state);
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
    if (flags & F_RESUME)
      diag_from_memory();
    else
      recompute(false);

    int64_t proposals = 0, accepts = 0, nonpos = 0, err = 0;
    double max_drift = 0.0;
    int recoveries = 0;

    if (d.op == OP_SWEEPS) {
      // running bin sums, loaded on entry to a bin and stored when it is left
      // or the launch ends (a chain split over launches sums like one launch)
      double gacc = 0.0, nacc_u = 0.0, nacc_d = 0.0, dacc = 0.0;
      int64_t cur_bin = -1;
      const int64_t nm = d.n_measure, nb = d.n_bins;
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
          append(l, fu, fd);
          if (kb >= kdepth) flush();
          flip_field(l);
          mark_flip(fl, l);
          proposals += l - l0 + 1;
          ++accepts;
          l0 = l + 1;
          l = scan(l0, uv, fu, fd, nonpos, err);
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
          const double dr = recompute(!retry);
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
        if (w >= d.n_warmup) {
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
          measure_green(gacc);
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
        append(l, du * recip(Ru), dd * recip(Rd));
        if (kb >= kdepth) flush();
        flip_field(l);
      }
      flush();
    } else if (d.op == OP_RECOMPUTE) {
      max_drift = recompute(true);
    }

    if ((flags & F_SAVE) && wave == 0) {  // G is already in its state area
      static_for<JW>([&](auto jj) __attribute__((always_inline)) {
        const int m = lane + 64 * jj;
        if (m < L) fields[m] = (int8_t)sv[jj];
      });
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
__global__ __launch_bounds__(C::NTH, 1) void sweep_global_kernel(const ImpDesc* __restrict__ descs,
                                                                 const int32_t* __restrict__ order, int n_items,
                                                                 int* __restrict__ queue, uint8_t* __restrict__ ws) {
  __shared__ GSmem<C> sm;
  EngineG<C> e(sm);
  for (;;) {
    if (threadIdx.x == 0) sm.item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = sm.item;
    __syncthreads();
    if (it >= n_items) break;
    e.run(descs + order[it], ws);
  }
}

template <int LT>
static KernelInfo ginfo() {
  using C = GCfg<LT>;
  return KernelInfo{LT, 0, 1, C::NTH, sizeof(GSmem<C>), reinterpret_cast<const void*>(&sweep_global_kernel<C>)};
}

static const KernelInfo kGlobal[] = {ginfo<80>(), ginfo<96>(), ginfo<112>(), ginfo<128>(), ginfo<144>(), ginfo<160>()};

int global_kernels(const KernelInfo** list) {
  *list = kGlobal;
  return (int)(sizeof(kGlobal) / sizeof(kGlobal[0]));
}

}  // namespace hfqmc
