// hfqmc_window.hip -- the fp64 window-update kernels (one instantiation per
// padded slice count and tile-rows per wave) and the window kernel registry.
#include "hfqmc_window.h"

namespace hfqmc {

static const KernelInfo kWindowFp64[] = {
    winfo<16, 1>(), winfo<32, 1>(), winfo<32, 2>(), winfo<48, 1>(), winfo<48, 3>(),
    winfo<64, 1>(), winfo<64, 2>(), winfo<80, 1>(), winfo<80, 5>(), winfo<96, 1>(), winfo<96, 3>(), winfo<128, 2>(), winfo<128, 4>(),
};

int window_kernels_fp64(const KernelInfo** list) {
  *list = kWindowFp64;
  return (int)(sizeof(kWindowFp64) / sizeof(kWindowFp64[0]));
}

// All window kernels, fp64 first.
int window_kernels(const KernelInfo** list) {
  static KernelInfo all[64];
  static int n = [] {
    int k = 0;
    const KernelInfo* l = nullptr;
    for (int part = 0; part < 2; ++part) {
      const int m = part == 0 ? window_kernels_fp64(&l) : window_kernels_mixed(&l);
      for (int i = 0; i < m && k < 64; ++i) all[k++] = l[i];
    }
    return k;
  }();
  *list = all;
  return n;
}

}  // namespace hfqmc
