// loglik_bf16.hip -- instantiations of the likelihood kernel for SPS_BF16X3,
// C <= 5 outcomes (C >= 6 live in loglik_bf16_wide.hip, a separate unit so
// the two compile in parallel).
#include "loglik_kernel.h"

namespace sps {

LoglikEntry lookup_bf16(int nc, int ks, int mode) {
#define SPS_E(NC, KS)                                                                          \
    if (nc == NC && ks == KS)                                                                  \
        return mode == MODE_GRAD     ? loglik_entry_bf16<NC, KS, MODE_GRAD>()                         \
               : mode == MODE_PEROBS ? loglik_entry_bf16<NC, KS, MODE_PEROBS>()                       \
                                     : loglik_entry_bf16<NC, KS, MODE_FWD>();
    SPS_E(1, 1)
    SPS_E(1, 2)
    SPS_E(1, 4)
    SPS_E(2, 1)
    SPS_E(2, 2)
    SPS_E(2, 4)
    SPS_E(3, 1)
    SPS_E(3, 2)
    SPS_E(3, 4)
    SPS_E(4, 1)
    SPS_E(4, 2)
    SPS_E(4, 4)
#undef SPS_E
    return lookup_bf16_wide(nc, ks, mode);
}

}  // namespace sps
