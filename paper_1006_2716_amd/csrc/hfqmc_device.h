// hfqmc_device.h -- device helpers shared by the gfx950 kernels of the
// Hirsch-Fye QMC engine (register-tile and global-memory sweep kernels).
// Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "hfqmc_internal.h"

namespace hfqmc {

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0..N-1, so
// every array index inside f is a constant before any optimisation runs and
// register arrays can never be demoted to scratch by a run-time index.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Compile-time case selection: f(std::integral_constant<int, idx>) for a
// run-time idx in [0, N), by a binary tree of uniform branches (depth
// log2 N instead of a chain of N compares); every leaf sees a constant.
template <int Lo, int Hi, class F>
__device__ __forceinline__ void dispatch_impl(int idx, F&& f) {
  if constexpr (Hi - Lo == 1) {
    f(std::integral_constant<int, Lo>{});
  } else {
    constexpr int Mid = (Lo + Hi) / 2;
    if (idx < Mid)
      dispatch_impl<Lo, Mid>(idx, f);
    else
      dispatch_impl<Mid, Hi>(idx, f);
  }
}
template <int N, class F>
__device__ __forceinline__ void dispatch(int idx, F&& f) {
  dispatch_impl<0, N>(idx, f);
}

// ------------------------------------------------------------- Philox4x64-10
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten
// rounds of two 64x64->128 multiplies, Weyl key schedule.
struct U64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, c0), lo0 = kM0 * c0;
    const uint64_t hi1 = __umul64hi(kM1, c2), lo1 = kM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return U64x4{{c0, c1, c2, c3}};
}

// Purposes of the Philox counter word 2.
constexpr uint64_t kPurposeInit = 1, kPurposeSweep = 2;

__device__ __forceinline__ double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// ------------------------------------------------------------- lane helpers
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int readlane_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

template <int JW, typename T>
__device__ __forceinline__ T pick(const T (&a)[JW], int jj) {
  T r = a[0];
  static_for<JW>([&](auto k) __attribute__((always_inline)) {
    if (k > 0 && jj == k) r = a[k];
  });
  return r;
}

// Reciprocal to full fp64 precision: hardware estimate plus two Newton steps.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Device memory seen as the global address space: loads and stores through
// these pointers are global_* instructions, not flat ones (which also count
// against the LDS wait counter).
typedef __attribute__((address_space(1))) double gdouble;

// Marks slice l in a uniform bit mask of JW words (slice m: word m / 64).
template <int JW>
__device__ __forceinline__ void mark_flip(uint64_t (&fl)[JW], int l) {
  static_for<JW>([&](auto jj) __attribute__((always_inline)) {
    if (jj == (l >> 6)) fl[jj] ^= 1ull << (l & 63);
  });
}

// Per-wave copy of an impurity's slice state: slice m lives in lane m % 64,
// word m / 64.  Every wave of the workgroup keeps its own copy and takes the
// same Metropolis decisions from it, so rejections need no communication.
template <int JW>
struct SliceState {
  double dgu[JW], dgd[JW];  // diagonals of G_up, G_dn
  double fpu[JW], fpd[JW];  // flip factors exp(-2 sigma lambda s_m) - 1 of the slices
  int sv[JW];               // fields s_m

  __device__ __forceinline__ void set_field(int jj, int s, double dflip_p, double dflip_m) {
    sv[jj] = s;
    fpu[jj] = s > 0 ? dflip_p : dflip_m;  // up:   exp(-2 lambda s) - 1
    fpd[jj] = s > 0 ? dflip_m : dflip_p;  // down: exp(+2 lambda s) - 1
  }

  __device__ __forceinline__ void flip_field(int l, int lane, double dflip_p, double dflip_m) {
    const int jj = l >> 6, ln = l & 63;
    if (lane == ln)
      static_for<JW>([&](auto k) __attribute__((always_inline)) {
        if (k == jj) set_field(k, -sv[k], dflip_p, dflip_m);
      });
  }

  // Vectorised Metropolis scan over slices [l0, L): rejections leave G
  // unchanged, so every remaining slice is tested against the current
  // diagonals at once (lane m tests slice m with exactly the arithmetic of a
  // sequential scan) and the first accepted slice is found by a wave ballot.
  // Returns that slice (L if none) and its factors f_s = d_s / R_s; counts
  // the rejected R <= 0 (never seen in exact arithmetic) into nonpos/err.
  __device__ __forceinline__ int scan(int l0, int L, int lane, const double (&uv)[JW], double& fu, double& fd,
                                      int64_t& nonpos, int64_t& err) const {
    uint64_t acc_mask[JW], bad_mask[JW];
    double Fu[JW], Fd[JW];
    static_for<JW>([&](auto jj) __attribute__((always_inline)) {
      const int m = lane + 64 * jj;
      const bool live = m >= l0 && m < L;
      const double Ru = __builtin_fma(1.0 - dgu[jj], fpu[jj], 1.0);
      const double Rd = __builtin_fma(1.0 - dgd[jj], fpd[jj], 1.0);
      const double R = Ru * Rd;
      acc_mask[jj] = __ballot(live && uv[jj] < R);
      bad_mask[jj] = __ballot(live && !(R > 0.0));
      // every lane forms its own factors d_s / R_s, off the critical path of
      // the ballot; the accepted lane's pair is read out below
      Fu[jj] = fpu[jj] * recip(Ru);
      Fd[jj] = fpd[jj] * recip(Rd);
      __asm__ volatile("" : "+v"(Fu[jj]), "+v"(Fd[jj]));  // computed before the exit test
    });
    int l = L;
    static_for<JW>([&](auto k) __attribute__((always_inline)) {
      constexpr int jj = JW - 1 - decltype(k)::value;  // highest word first, lowest wins
      if (acc_mask[jj]) l = 64 * jj + __builtin_ctzll(acc_mask[jj]);
    });
    static_for<JW>([&](auto jj) __attribute__((always_inline)) {
      const int hi = l - 64 * jj;  // slices below l were rejected
      const uint64_t below = hi >= 64 ? ~0ull : (hi <= 0 ? 0ull : ((1ull << hi) - 1));
      const uint64_t bad = bad_mask[jj] & below;
      nonpos += __builtin_popcountll(bad);
      if (bad) err = 1;
    });
    const int ls = l < L ? l : 0, jj = ls >> 6, ln = ls & 63;
    fu = readlane_d(pick<JW>(Fu, jj), ln);
    fd = readlane_d(pick<JW>(Fd, jj), ln);
    return l;
  }
};

// One compiled sweep kernel.  RT = tile-rows per wave of the register-tile
// kernels, 0 for the global-memory kernel; DK = update kind (0 rank-one,
// 1 delayed fp64, 2 delayed with fp32 products, 3 window updates, 4 window
// updates with fp32 products).
struct KernelInfo {
  int LT, RT, DK, threads;
  size_t lds;
  const void* fn;
};

// Kernels of the other translation units.
int global_kernels(const KernelInfo** list);
int window_kernels(const KernelInfo** list);
int window_global_kernels(const KernelInfo** list);

}  // namespace hfqmc
