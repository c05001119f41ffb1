// loglik_pipe_fwd_c.hip -- instantiations of the pipelined BF16x3 likelihood kernel
// (forward only), C = 6 outcomes, k > 32.
#include "loglik_pipe.h"

namespace sps {

LoglikEntry lookup_pipe_fwd_c(int nc, int ks) {
    if (nc == 5 && ks == 2) return loglik_pipe_entry<5, 2, false>();
    if (nc == 5 && ks == 4) return loglik_pipe_entry<5, 4, false>();
    return LoglikEntry{};
}

}  // namespace sps
