// loglik_pipe_fwd_b.hip -- instantiations of the pipelined BF16x3 likelihood kernel
// (forward only), C = 4..5 outcomes, k > 32.
#include "loglik_pipe.h"

namespace sps {

LoglikEntry lookup_pipe_fwd_b(int nc, int ks) {
    if (nc == 3 && ks == 2) return loglik_pipe_entry<3, 2, false>();
    if (nc == 3 && ks == 4) return loglik_pipe_entry<3, 4, false>();
    if (nc == 4 && ks == 2) return loglik_pipe_entry<4, 2, false>();
    if (nc == 4 && ks == 4) return loglik_pipe_entry<4, 4, false>();
    return LoglikEntry{};
}

}  // namespace sps
