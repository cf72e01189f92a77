// hfqmc_lattice.h -- descriptors of the lattice self-consistency kernels
// (Eq. (2) and the impurity Dyson equation), shared by the host ABI and the
// gfx950 kernels.  Not part of the public C ABI.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace hfqmc {

// ---- lattice self-consistency (Eq. (2) and the impurity Dyson equation) ----
// Complex arrays are (re, im) pairs; "spin-frequency-site" arrays are laid
// out [spin][n][site] with n the Matsubara index, w_n = (2n + 1) pi / beta.

constexpr int kMaxLayer = 64;     // sites per layer of the lattice kernel
constexpr int kMaxFreq = 2048;    // Matsubara frequencies per call

// One call of the layered lattice Green function: diag of
// [(i w_n + mu) 1 - hop - diag(eps_s) - diag(sigma_s(i w_n))]^-1 for every
// spin s and frequency n, hop block tridiagonal over layers of `layer` sites
// with diagonal couplings between neighbouring layers.
struct LatDesc {
  int32_t n_sites, layer, n_layers, n_freq;
  double beta, mu;
  const double* blocks;    // n_layers blocks layer x layer (row-major) of hop
  const double* coupling;  // (n_layers - 1) x layer: hop(site j of layer k, site j of layer k + 1)
  const double* eps;       // 2 x n_sites
  const double* sigma;     // spin-frequency-site, complex
  double* gloc;            // spin-frequency-site, complex (output)
  double* work;            // per (spin, n): n_layers padded blocks of the left-connected inverses
};

// Weiss functions of selected sites: W = (G_loc^-1 + sigma)^-1 on the
// Matsubara grid, and the solver's samples g(tau_l) = -W(tau_l), l < L.
struct WeissDesc {
  int32_t n_sites, n_freq, L, n_sel;
  double beta, mu;
  const double* eps;       // 2 x n_sites
  const double* gloc;      // spin-frequency-site, complex
  const double* sigma;     // spin-frequency-site, complex
  const int32_t* sites;    // n_sel site indices
  double* weiss_iw;        // [spin][n][j], complex (output)
  double* weiss_tau;       // [j][spin][l], l < L (output)
};

// Self-energy of selected sites from the solver's g(tau_k), k = 0 .. L, and
// densities; sigma <- mix sigma_new + (1 - mix) sigma at those sites.
struct SigmaDesc {
  int32_t n_sites, n_freq, L, n_sel;
  double beta, mu, U, mix;
  const double* eps;       // 2 x n_sites
  const int32_t* sites;    // n_sel site indices
  const double* weiss_iw;  // [spin][n][j], complex
  const double* gimp_tau;  // [j][spin][k], k <= L
  const double* density;   // [j][spin]
  double* sigma;           // spin-frequency-site, complex (updated in place)
};

// Padded layer width of the lattice kernel for `layer` sites.
inline int lattice_pad(int layer) { return layer <= 16 ? 16 : layer <= 32 ? 32 : layer <= 48 ? 48 : 64; }

}  // namespace hfqmc
