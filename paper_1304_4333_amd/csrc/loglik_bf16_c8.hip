// loglik_bf16_c8.hip -- instantiations of the likelihood kernel for
// SPS_BF16X3 with C = 8 outcomes (seven outcome chains per wave; the largest
// register footprint, compiled with the default MFMA register assignment).
#include "loglik_kernel.h"

namespace sps {

LoglikEntry lookup_bf16_c8(int nc, int ks, int mode) {
#define SPS_E(NC, KS)                                                                          \
    if (nc == NC && ks == KS)                                                                  \
        return mode == MODE_GRAD     ? loglik_entry_bf16<NC, KS, MODE_GRAD>()                         \
               : mode == MODE_PEROBS ? loglik_entry_bf16<NC, KS, MODE_PEROBS>()                       \
                                     : loglik_entry_bf16<NC, KS, MODE_FWD>();
    SPS_E(7, 1)
    SPS_E(7, 2)
    SPS_E(7, 4)
#undef SPS_E
    return LoglikEntry{};
}

}  // namespace sps
