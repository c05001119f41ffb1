// loglik_pipe_fwd_d.hip -- instantiations of the pipelined BF16x3 likelihood kernel
// (forward only), C = 7..8 outcomes, k > 32.
#include "loglik_pipe.h"

namespace sps {

LoglikEntry lookup_pipe_fwd_d(int nc, int ks) {
    if (nc == 6 && ks == 2) return loglik_pipe_entry<6, 2, false>();
    if (nc == 6 && ks == 4) return loglik_pipe_entry<6, 4, false>();
    if (nc == 7 && ks == 2) return loglik_pipe_entry<7, 2, false>();
    if (nc == 7 && ks == 4) return loglik_pipe_entry<7, 4, false>();
    return LoglikEntry{};
}

}  // namespace sps
