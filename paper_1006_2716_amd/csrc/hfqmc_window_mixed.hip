// hfqmc_window_mixed.hip -- window-update kernels whose window flush forms
// fp32 products (v_mfma_f32_16x16x4f32) added into the fp64 tiles.  None
// at 128 slices: the conversions and adds of the fp32 products push the
// two-waves-per-SIMD shape into scratch, and the fp64 kernel serves there.
#include "hfqmc_window.h"

namespace hfqmc {

static const KernelInfo kWindowMixed[] = {
    winfo<32, 1, 1>(), winfo<48, 1, 1>(), winfo<48, 3, 1>(), winfo<64, 2, 1>(), winfo<80, 1, 1>(), winfo<96, 1, 1>(),
};

int window_kernels_mixed(const KernelInfo** list) {
  *list = kWindowMixed;
  return (int)(sizeof(kWindowMixed) / sizeof(kWindowMixed[0]));
}

}  // namespace hfqmc
