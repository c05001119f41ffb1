// loglik_bf16_wide.hip -- instantiations of the likelihood kernel for
// SPS_BF16X3 with C = 6 or 7 outcomes (five or six outcome chains per wave);
// C = 8 lives in loglik_bf16_c8.hip.
#include "loglik_kernel.h"

namespace sps {

LoglikEntry lookup_bf16_wide(int nc, int ks, int mode) {
#define SPS_E(NC, KS)                                                                          \
    if (nc == NC && ks == KS)                                                                  \
        return mode == MODE_GRAD     ? loglik_entry_bf16<NC, KS, MODE_GRAD>()                         \
               : mode == MODE_PEROBS ? loglik_entry_bf16<NC, KS, MODE_PEROBS>()                       \
                                     : loglik_entry_bf16<NC, KS, MODE_FWD>();
    SPS_E(5, 1)
    SPS_E(5, 2)
    SPS_E(5, 4)
    SPS_E(6, 1)
    SPS_E(6, 2)
    SPS_E(6, 4)
#undef SPS_E
    return lookup_bf16_c8(nc, ks, mode);
}

}  // namespace sps
