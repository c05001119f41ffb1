// loglik_fp64.hip -- instantiations of the likelihood kernel for SPS_FP64.
#include "loglik_kernel.h"

namespace sps {

LoglikEntry lookup_fp64(int nc, int ks, int mode) {
#define SPS_E(NC, KS)                                                                          \
    if (nc == NC && ks == KS)                                                                  \
        return mode == MODE_GRAD     ? loglik_entry<SPS_FP64, NC, KS, MODE_GRAD>()                  \
               : mode == MODE_PEROBS ? loglik_entry<SPS_FP64, NC, KS, MODE_PEROBS>()                \
                                     : loglik_entry<SPS_FP64, NC, KS, MODE_FWD>();
    SPS_E(1, 4)
    SPS_E(1, 8)
    SPS_E(1, 16)
    SPS_E(1, 32)
    SPS_E(2, 4)
    SPS_E(2, 8)
    SPS_E(2, 16)
    SPS_E(2, 32)
    SPS_E(3, 4)
    SPS_E(3, 8)
    SPS_E(3, 16)
    SPS_E(3, 32)
    SPS_E(4, 4)
    SPS_E(4, 8)
    SPS_E(4, 16)
    SPS_E(4, 32)
    SPS_E(5, 4)
    SPS_E(5, 8)
    SPS_E(5, 16)
    SPS_E(5, 32)
    SPS_E(6, 4)
    SPS_E(6, 8)
    SPS_E(6, 16)
    SPS_E(6, 32)
    SPS_E(7, 4)
    SPS_E(7, 8)
    SPS_E(7, 16)
    SPS_E(7, 32)
#undef SPS_E
    return LoglikEntry{};
}

}  // namespace sps
