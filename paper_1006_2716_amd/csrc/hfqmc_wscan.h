// hfqmc_wscan.h -- the decisions of one 16-slice window, taken by one wave
// on the two 16 x 16 diagonal blocks G_s[W,W] (shared by the window-update
// kernels that keep G in registers and in device memory).
//
// Lane (q, c) = (lane / 16, lane % 16) holds rows 4q + r, r = 0..3, of block
// column c.  Every proposal of the window reads only the block diagonal
// (R_s = 1 + (1 - G_s[l][l]) d_s, Eq. (1) and the Hirsch-Fye ratio of the
// "Model and Methods" section), and an accepted flip changes the block by a
// rank-one term built from the block itself, so the whole window runs in
// registers: no barrier and no memory traffic per accept.
#pragma once
#include "hfqmc_device.h"

namespace hfqmc {

typedef double wd4 __attribute__((ext_vector_type(4)));
typedef float wf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double bperm_d(int addr, double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// a[k] for a per-lane k in [0, 4).  The array is taken by value: a select
// of element addresses would turn register arrays into scratch memory.
struct D4 {
  double v[4];
};
__device__ __forceinline__ double sel4(D4 a, int k) {
  const double x = (k & 1) ? a.v[1] : a.v[0];
  const double y = (k & 1) ? a.v[3] : a.v[2];
  return (k & 2) ? y : x;
}
__device__ __forceinline__ D4 d4of(const double (&a)[4]) { return D4{{a[0], a[1], a[2], a[3]}}; }

enum WinMode : int {
  WM_METROPOLIS = 0,  // Metropolis decisions over the window's slices
  WM_DYSON = 1,       // switch every slice's potential on from V = 0
  WM_FORCE = 2,       // flip one given slice
};

// Rank-one update of both window blocks and of Q for an accepted slice j
// with factors f_s.  The wave keeps B'_s = B_s - 1 and Q'_s = Q_s - 1, so
// column j of B' is already B_s[:,j] - e_j: u_s = f_s B'_s[:,j],
// B'_s += u_s B_s[j,:], Q'_s += u_s Q_s[j,:] (rows of B and Q: the primed
// rows plus e_j).  Column j comes from lane 16q + j, row j from lane
// 16(j/4) + c, register j % 4 (a uniform choice: four branch leaves).
__device__ __forceinline__ void win_rank1(int lane, int c, int j, double fu, double fd, double (&bu)[4],
                                          double (&bd)[4], double (&qu)[4], double (&qd)[4]) {
  const int src_col = ((lane & 48) | j) << 2;
  const int src_row = (((j & 12) << 2) | c) << 2;
  // the column first: its permutes do not wait for the row's branch
  double cu[4], cd[4];
  static_for<4>([&](auto r) __attribute__((always_inline)) {
    cu[r] = bperm_d(src_col, bu[r]);
    cd[r] = bperm_d(src_col, bd[r]);
  });
  double rbu = 0.0, rbd = 0.0, rqu = 0.0, rqd = 0.0;
  dispatch<4>(j & 3, [&](auto jr) __attribute__((always_inline)) {
    constexpr int R = decltype(jr)::value;
    rbu = bperm_d(src_row, bu[R]);
    rbd = bperm_d(src_row, bd[R]);
    rqu = bperm_d(src_row, qu[R]);
    rqd = bperm_d(src_row, qd[R]);
  });
  const double e = c == j ? 1.0 : 0.0;
  rbu += e;
  rbd += e;
  rqu += e;
  rqd += e;
  static_for<4>([&](auto r) __attribute__((always_inline)) {
    const double au = fu * cu[r], ad = fd * cd[r];
    bu[r] = __builtin_fma(au, rbu, bu[r]);
    bd[r] = __builtin_fma(ad, rbd, bd[r]);
    qu[r] = __builtin_fma(au, rqu, qu[r]);
    qd[r] = __builtin_fma(ad, rqd, qd[r]);
  });
}

// The window's decisions, on one wave.  ru, rd point at this lane's first
// element (block row 4q, column c) of the window's diagonal blocks of G_up,
// G_dn, rows rs doubles apart.  fw0: the window's fields (bit i set <=>
// s = -1 on slice base + i); fa, fb: the factors d_s for sigma s_l = +1 and
// -1 (flip factors, or exp(V) - 1 for the Dyson mode); u: the uniform of
// slice base + c (Metropolis mode); jf: the slice of the force mode; px:
// test hook, NaN poisons the blocks.  Lane (q, c) with q == c/4 is the
// diagonal lane of window slice c (it holds B'_s[c][c] in register c % 4).
// Writes P_s = D_s Q_s (window coordinates, rows TS apart) to pu, pd and S,
// |S| (bit 8: a ratio that was not a positive number) and the accepted
// slices in increasing order (4 bits each) to win[0..3]; counts accepts and
// non-positive ratios (Metropolis mode).
template <int TS>
__device__ __forceinline__ void win_scan(const double* ru, const double* rd, int rs, int lane, int q, int c,
                                         int base, int L, uint32_t fw0, double fa, double fb, int mode, int jf,
                                         double u, double px, double* ratio_out, double* pu, double* pd,
                                         uint32_t* win, int64_t& accepts, int64_t& nonpos, int64_t& err) {
  double bu[4], bd[4], qu[4], qd[4];
  static_for<4>([&](auto r) __attribute__((always_inline)) {
    const double e = (4 * q + r == c) ? 1.0 : 0.0;
    bu[r] = (ru[r * rs] - e) * px;
    bd[r] = (rd[r * rs] - e) * px;
    qu[r] = qd[r] = 0.0;
  });
  const bool dl = q == (c >> 2);
  const int rr = c & 3;
  const bool in = base + c < L;
  const int sn = (fw0 >> c) & 1;
  const double du = sn ? fb : fa, dd = sn ? fa : fb;
  uint32_t S = 0;
  uint64_t slist = 0, badmask = 0;
  int m = 0, l0 = 0;
  for (;;) {
    // R_s = 1 + (1 - G_s[c][c]) d_s = 1 - B'_s[c][c] d_s
    const double Ru = __builtin_fma(-sel4(d4of(bu), rr), du, 1.0);
    const double Rd = __builtin_fma(-sel4(d4of(bd), rr), dd, 1.0);
    const double R = Ru * Rd;
    const bool live = dl && in && c >= l0 && (mode != WM_FORCE || c == jf);
    const uint64_t acc = __ballot(live && (mode != WM_METROPOLIS || u < R));
    double Fu = du * recip(Ru), Fd = dd * recip(Rd);
    // kept ahead of the loop exit: the reciprocals overlap the ballot instead
    // of following it on the path to the next accept
    __asm__ volatile("" : "+v"(Fu), "+v"(Fd));
    if (mode == WM_METROPOLIS) {
      // R <= 0 (or not a number) among the slices this step rejects: every
      // slice is rejected at most once, so the lanes can be collected
      const uint64_t below = acc ? ((1ull << __builtin_ctzll(acc)) - 1) : ~0ull;
      badmask |= __ballot(live && !(R > 0.0)) & below;
    }
    if (!acc) break;
    const int lj = __builtin_ctzll(acc), j = lj & 15;
    const double fu = readlane_d(Fu, lj), fd = readlane_d(Fd, lj);
    if (mode == WM_FORCE) {
      const double rv = readlane_d(R, lj);
      if (lane == 0 && ratio_out) *ratio_out = rv;
    }
    win_rank1(lane, c, j, fu, fd, bu, bd, qu, qd);
    S |= 1u << j;
    slist |= (uint64_t)j << (4 * m);
    ++m;
    l0 = j + 1;
  }
  // P_s = D_s Q_s: row i scaled by the factor of slice i if accepted, else 0
  pu += (4 * q) * TS + c;
  pd += (4 * q) * TS + c;
  static_for<4>([&](auto r) __attribute__((always_inline)) {
    const int i = 4 * q + r;
    const int si = (fw0 >> i) & 1;
    const bool acc_i = (S >> i) & 1;
    const double fu_i = si ? fb : fa, fd_i = si ? fa : fb;
    const double e = i == c ? 1.0 : 0.0;
    pu[r * TS] = acc_i ? fu_i * (qu[r] + e) : 0.0;
    pd[r * TS] = acc_i ? fd_i * (qd[r] + e) : 0.0;
  });
  if (mode == WM_METROPOLIS) {
    accepts += m;
    nonpos += __builtin_popcountll(badmask);
    if (badmask) err = 1;
  }
  if (lane == 0) {
    win[0] = S;
    win[1] = (uint32_t)m | (badmask ? 0x100u : 0u);
    win[2] = (uint32_t)slist;
    win[3] = (uint32_t)(slist >> 32);
  }
}

}  // namespace hfqmc
