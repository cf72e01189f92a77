// hfqmc_lattice.hip -- gfx950 kernels of the real-space DMFT self-consistency
// around the impurity solver.
//
// rgf_kernel     the lattice Dyson equation, Eq. (2): the site-diagonal part of
//                [(i w_n + mu) 1 - hop - diag(eps_s) - diag(sigma_s(i w_n))]^-1
//                for every spin and Matsubara frequency, one workgroup per
//                (spin, frequency).  With the sites ordered layer by layer and
//                nearest-neighbour hopping (a square lattice row by row), the
//                matrix is block tridiagonal with diagonal couplings c_k between
//                layers, and its diagonal follows exactly from the recursive
//                Green function sweep (block Gaussian elimination):
//                  forward   g_0 = A_0^-1,  g_k = (A_k - C_k-1 g_k-1 C_k-1)^-1
//                  backward  G_last = g_last,  G_k = g_k + X_k G_k+1 X_k^T,
//                            X_k = g_k C_k
//                with C_k = diag(c_k) and every g_k, G_k complex symmetric.
//                Cost O(N layer^2) instead of the O(N^3) of a dense inverse.
//                Blocks are inverted by Gauss-Jordan elimination without
//                pivoting: every block has a positive definite imaginary part
//                (w_n - Im sigma > 0, and Schur complements keep it), so no
//                pivot vanishes.
// weiss_kernel   W = (G_loc^-1 + sigma)^-1 and its samples g(tau_l) for the
//                solver: the level 1 / (i w - e) exactly, the rest by the
//                Matsubara sum over the kept frequencies and their negatives.
// sigma_kernel   the self-energy from the solver's g(tau_k): the
//                Hartree-shifted Weiss function exactly plus the transform of
//                the piecewise-linear interpolant of the difference, below
//                w_n dtau = pi / 2; the two-moment tail above.
#include <math.h>

#include "hfqmc_internal.h"
#include "hfqmc_lattice.h"

namespace hfqmc {

namespace {

struct cplx {
  double re, im;
};

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {__builtin_fma(a.re, b.re, -a.im * b.im), __builtin_fma(a.re, b.im, a.im * b.re)};
}
// a - b c
__device__ __forceinline__ cplx cfms(cplx a, cplx b, cplx c) {
  return {a.re - __builtin_fma(b.re, c.re, -b.im * c.im), a.im - __builtin_fma(b.re, c.im, b.im * c.re)};
}
// a + b c
__device__ __forceinline__ cplx cfma(cplx a, cplx b, cplx c) {
  return {a.re + __builtin_fma(b.re, c.re, -b.im * c.im), a.im + __builtin_fma(b.re, c.im, b.im * c.re)};
}
__device__ __forceinline__ cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ cplx cinv(cplx a) {
  const double d = __builtin_fma(a.re, a.re, a.im * a.im);
  return {a.re / d, -a.im / d};
}

// g(tau) of the single level e (the transform of 1 / (i w - e)), 0 <= tau <= beta,
// with non-positive exponents only.
__device__ double level_tau(double e, double beta, double tau) {
  return e >= 0.0 ? exp(-e * tau) / (1.0 + exp(-beta * e)) : exp(e * (beta - tau)) / (exp(beta * e) + 1.0);
}

// -(2 / beta) sum_n Re[exp(-i w_n tau_l) r_n] for tau_l = l beta / L: the phase
// (2n + 1) l pi / L is reduced exactly in integers (modulo 2L).
__device__ double matsubara_rest(const cplx* r, int nf, int l, int L, double beta) {
  double acc = 0.0;
  int m = l % (2 * L);  // (2n + 1) l mod 2L at n = 0
  const int step = (2 * l) % (2 * L);
  for (int n = 0; n < nf; ++n) {
    double sn, cs;
    sincospi((double)m / (double)L, &sn, &cs);
    acc += __builtin_fma(cs, r[n].re, sn * r[n].im);  // Re[(cs - i sn) r]
    m += step;
    if (m >= 2 * L) m -= 2 * L;
  }
  return -(2.0 / beta) * acc;
}

}  // namespace

// ------------------------------------------------------------ lattice Green

template <int BP>
__global__ __launch_bounds__(256) void rgf_kernel(LatDesc d) {
  constexpr int R = BP / 16;   // each thread owns rows ty + 16a, columns tx + 16c
  constexpr int LD = BP + 1;   // padded row stride of the LDS blocks
  __shared__ cplx S[BP * LD];  // G_k+1 / Y during the backward sweep
  __shared__ cplx X[BP * LD];  // X_k; pivot row and column during elimination
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
  const int mat = blockIdx.x;  // spin * n_freq + n
  const int s = mat / d.n_freq, n = mat % d.n_freq;
  const int b = d.layer, nl = d.n_layers, N = d.n_sites;
  const double w = (2.0 * n + 1.0) * M_PI / d.beta;
  const double* eps = d.eps + (size_t)s * N;
  const cplx* sig = reinterpret_cast<const cplx*>(d.sigma) + ((size_t)s * d.n_freq + n) * N;
  cplx* out = reinterpret_cast<cplx*>(d.gloc) + ((size_t)s * d.n_freq + n) * N;
  cplx* ws = reinterpret_cast<cplx*>(d.work) + (size_t)mat * nl * BP * BP;
  cplx M[R][R];

  // ---- forward: left-connected inverses g_k, kept in registers, stored to ws
  for (int k = 0; k < nl; ++k) {
    const int base = k * b;
    const double* blk = d.blocks + (size_t)k * b * b;
    const double* cprev = k > 0 ? d.coupling + (size_t)(k - 1) * b : nullptr;
#pragma unroll
    for (int a = 0; a < R; ++a) {
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const int i = ty + 16 * a, j = tx + 16 * c;
        cplx v = {i == j ? 1.0 : 0.0, 0.0};  // padding: identity
        if (i < b && j < b) {
          const double h = blk[i * b + j];
          v = {-h, 0.0};
          if (i == j) {
            const cplx sg = sig[base + i];
            v = {d.mu - h - eps[base + i] - sg.re, w - sg.im};
          }
          if (k > 0) v = csub(v, cscale(M[a][c], cprev[i] * cprev[j]));
        }
        M[a][c] = v;
      }
    }
    // Gauss-Jordan elimination in registers; row and column p go through LDS
    // (double-buffered by the parity of p, one barrier per pivot)
    for (int p = 0; p < b; ++p) {
      cplx* rb = X + (p & 1) * 2 * BP;
      cplx* cb = rb + BP;
      const int pa = p >> 4, pt = p & 15;
      // row p is held by the threads with ty = p % 16 in their register row
      // p / 16, column p by those with tx = p % 16 in register column p / 16
      // (register indices stay compile-time constants)
#pragma unroll
      for (int a = 0; a < R; ++a)
        if (a == pa && ty == pt) {
#pragma unroll
          for (int c = 0; c < R; ++c) rb[tx + 16 * c] = M[a][c];
        }
#pragma unroll
      for (int c = 0; c < R; ++c)
        if (c == pa && tx == pt) {
#pragma unroll
          for (int a = 0; a < R; ++a) cb[ty + 16 * a] = M[a][c];
        }
      __syncthreads();
      const cplx piv = cinv(rb[p]);
      cplx f[R], r[R];
#pragma unroll
      for (int a = 0; a < R; ++a) f[a] = cmul(cb[ty + 16 * a], piv);
#pragma unroll
      for (int c = 0; c < R; ++c) r[c] = rb[tx + 16 * c];
#pragma unroll
      for (int a = 0; a < R; ++a) {
#pragma unroll
        for (int c = 0; c < R; ++c) {
          const int i = ty + 16 * a, j = tx + 16 * c;
          if (i == p)
            M[a][c] = j == p ? piv : cmul(r[c], piv);
          else if (j == p)
            M[a][c] = {-f[a].re, -f[a].im};
          else
            M[a][c] = cfms(M[a][c], f[a], r[c]);
        }
      }
    }
    cplx* gk = ws + (size_t)k * BP * BP;
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int c = 0; c < R; ++c) gk[(ty + 16 * a) * BP + tx + 16 * c] = M[a][c];
    __syncthreads();  // the pivot buffers are rewritten by the next layer
  }

  // ---- backward: G_k = g_k + X_k G_k+1 X_k^T, X_k = g_k diag(c_k)
#pragma unroll
  for (int a = 0; a < R; ++a)
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const int i = ty + 16 * a, j = tx + 16 * c;
      S[i * LD + j] = M[a][c];
      if (i == j && i < b) out[(nl - 1) * b + i] = M[a][c];
    }
  for (int k = nl - 2; k >= 0; --k) {
    const cplx* gk = ws + (size_t)k * BP * BP;
    const double* ck = d.coupling + (size_t)k * b;
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const int i = ty + 16 * a, j = tx + 16 * c;
        M[a][c] = gk[i * BP + j];
        X[i * LD + j] = cscale(M[a][c], j < b ? ck[j] : 0.0);
      }
    __syncthreads();
    cplx acc[R][R];
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int c = 0; c < R; ++c) acc[a][c] = {0.0, 0.0};
    for (int m = 0; m < b; ++m) {  // Y = X G (columns of X beyond b are zero)
      cplx xa[R], gc[R];
#pragma unroll
      for (int a = 0; a < R; ++a) xa[a] = X[(ty + 16 * a) * LD + m];
#pragma unroll
      for (int c = 0; c < R; ++c) gc[c] = S[m * LD + tx + 16 * c];
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int c = 0; c < R; ++c) acc[a][c] = cfma(acc[a][c], xa[a], gc[c]);
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int c = 0; c < R; ++c) {
        S[(ty + 16 * a) * LD + tx + 16 * c] = acc[a][c];
        acc[a][c] = {0.0, 0.0};
      }
    __syncthreads();
    for (int m = 0; m < b; ++m) {  // G_k = g_k + Y X^T
      cplx ya[R], xc[R];
#pragma unroll
      for (int a = 0; a < R; ++a) ya[a] = S[(ty + 16 * a) * LD + m];
#pragma unroll
      for (int c = 0; c < R; ++c) xc[c] = X[(tx + 16 * c) * LD + m];
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int c = 0; c < R; ++c) acc[a][c] = cfma(acc[a][c], ya[a], xc[c]);
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const int i = ty + 16 * a, j = tx + 16 * c;
        const cplx g = cadd(M[a][c], acc[a][c]);
        S[i * LD + j] = g;
        if (i == j && i < b) out[k * b + i] = g;
      }
    __syncthreads();
  }
}

// ------------------------------------------------------------ Weiss function

__global__ __launch_bounds__(256) void weiss_kernel(WeissDesc d) {
  extern __shared__ cplx rest[];  // n_freq
  const int j = blockIdx.x >> 1, s = blockIdx.x & 1;
  const int i = d.sites[j], N = d.n_sites, nf = d.n_freq;
  const double e = d.eps[(size_t)s * N + i] - d.mu;
  const cplx* gl = reinterpret_cast<const cplx*>(d.gloc) + (size_t)s * nf * N + i;
  const cplx* sg = reinterpret_cast<const cplx*>(d.sigma) + (size_t)s * nf * N + i;
  cplx* wout = reinterpret_cast<cplx*>(d.weiss_iw) + (size_t)s * nf * d.n_sel + j;
  for (int n = threadIdx.x; n < nf; n += blockDim.x) {
    const double w = (2.0 * n + 1.0) * M_PI / d.beta;
    const cplx W = cinv(cadd(cinv(gl[(size_t)n * N]), sg[(size_t)n * N]));
    wout[(size_t)n * d.n_sel] = W;
    rest[n] = csub(W, cinv({-e, w}));
  }
  __syncthreads();
  for (int l = threadIdx.x; l < d.L; l += blockDim.x) {
    const double tau = d.beta * l / d.L;
    d.weiss_tau[((size_t)j * 2 + s) * d.L + l] = level_tau(e, d.beta, tau) + matsubara_rest(rest, nf, l, d.L, d.beta);
  }
}

// ------------------------------------------------------------ self-energy

__global__ __launch_bounds__(256) void sigma_kernel(SigmaDesc d) {
  extern __shared__ cplx rest[];  // n_freq, then L + 1 doubles of the difference
  double* diff = reinterpret_cast<double*>(rest + d.n_freq);
  const int j = blockIdx.x >> 1, s = blockIdx.x & 1;
  const int i = d.sites[j], N = d.n_sites, nf = d.n_freq, L = d.L;
  const double e = d.eps[(size_t)s * N + i] - d.mu;
  const double n_other = d.density[(size_t)j * 2 + (1 - s)];
  const double s_inf = d.U * (n_other - 0.5);
  const double eh = e + s_inf;
  const cplx* win = reinterpret_cast<const cplx*>(d.weiss_iw) + (size_t)s * nf * d.n_sel + j;
  for (int n = threadIdx.x; n < nf; n += blockDim.x) {
    const double w = (2.0 * n + 1.0) * M_PI / d.beta;
    const cplx W = win[(size_t)n * d.n_sel];
    const cplx WH = cinv({cinv(W).re - s_inf, cinv(W).im});
    rest[n] = csub(WH, cinv({-eh, w}));
  }
  __syncthreads();
  const double* gi = d.gimp_tau + ((size_t)j * 2 + s) * (L + 1);
  for (int k = threadIdx.x; k <= L; k += blockDim.x) {
    const double tau = d.beta * k / L;
    diff[k] = gi[k] - (level_tau(eh, d.beta, tau) + matsubara_rest(rest, nf, k, L, d.beta));
  }
  __syncthreads();
  const int nc = L / 4 > 1 ? L / 4 : 1;
  const double dt = d.beta / L;
  cplx* sg = reinterpret_cast<cplx*>(d.sigma) + (size_t)s * nf * N + i;
  for (int n = threadIdx.x; n < nf; n += blockDim.x) {
    const double w = (2.0 * n + 1.0) * M_PI / d.beta;
    const cplx W = win[(size_t)n * d.n_sel];
    cplx snew;
    if (n < nc) {
      // weights of the hat functions: interior e^{i k th} 4 sin^2(th/2) / (w^2 dt),
      // ends i / w + (1 - e^{i th}) / (w^2 dt) and i / w - (1 - e^{-i th}) / (w^2 dt)
      double sh, ch, st, ct;
      sincospi((2.0 * n + 1.0) / (2.0 * L), &sh, &ch);
      sincospi((2.0 * n + 1.0) / L, &st, &ct);
      const double q = 1.0 / (w * w * dt);
      const double s2 = 2.0 * sh * sh;  // 1 - cos th
      cplx F = {diff[0] * s2 * q, diff[0] * (1.0 / w - st * q)};
      F = cadd(F, {-diff[L] * s2 * q, diff[L] * (1.0 / w - st * q)});
      const double wi = 2.0 * s2 * q;
      int m = 0;
      const int step = (2 * n + 1) % (2 * L);
      for (int k = 1; k < L; ++k) {
        m += step;
        if (m >= 2 * L) m -= 2 * L;
        double sk, ck;
        sincospi((double)m / (double)L, &sk, &ck);
        F.re = __builtin_fma(diff[k] * wi, ck, F.re);
        F.im = __builtin_fma(diff[k] * wi, sk, F.im);
      }
      const cplx iW = cinv(W);
      const cplx WH = cinv({iW.re - s_inf, iW.im});
      const cplx Gimp = csub(WH, F);
      snew = csub(iW, cinv(Gimp));
    } else {
      snew = {s_inf, -d.U * d.U * n_other * (1.0 - n_other) / w};
    }
    const cplx old = sg[(size_t)n * N];
    sg[(size_t)n * N] = cadd(cscale(snew, d.mix), cscale(old, 1.0 - d.mix));
  }
}

// ------------------------------------------------------------ launchers

size_t lattice_work_bytes(int layer, int n_layers, int n_freq) {
  const size_t bp = (size_t)lattice_pad(layer);
  return 2 * (size_t)n_freq * n_layers * bp * bp * sizeof(cplx);
}

hipError_t launch_lattice_green(const LatDesc& d, hipStream_t st) {
  const dim3 grid(2 * d.n_freq), block(256);
  switch (lattice_pad(d.layer)) {
    case 16: hipLaunchKernelGGL(rgf_kernel<16>, grid, block, 0, st, d); break;
    case 32: hipLaunchKernelGGL(rgf_kernel<32>, grid, block, 0, st, d); break;
    case 48: hipLaunchKernelGGL(rgf_kernel<48>, grid, block, 0, st, d); break;
    default: hipLaunchKernelGGL(rgf_kernel<64>, grid, block, 0, st, d); break;
  }
  return hipGetLastError();
}

hipError_t launch_weiss(const WeissDesc& d, hipStream_t st) {
  hipLaunchKernelGGL(weiss_kernel, dim3(2 * d.n_sel), dim3(256), sizeof(cplx) * d.n_freq, st, d);
  return hipGetLastError();
}

hipError_t launch_sigma(const SigmaDesc& d, hipStream_t st) {
  const size_t lds = sizeof(cplx) * d.n_freq + sizeof(double) * (d.L + 1);
  hipLaunchKernelGGL(sigma_kernel, dim3(2 * d.n_sel), dim3(256), lds, st, d);
  return hipGetLastError();
}

}  // namespace hfqmc
