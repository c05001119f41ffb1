// loglik_pipe_fwd_a.hip -- instantiations of the pipelined BF16x3 likelihood kernel
// (forward only), C = 2..3 outcomes, k > 32.
#include "loglik_pipe.h"

namespace sps {

LoglikEntry lookup_pipe_fwd_a(int nc, int ks) {
    if (nc == 1 && ks == 2) return loglik_pipe_entry<1, 2, false>();
    if (nc == 1 && ks == 4) return loglik_pipe_entry<1, 4, false>();
    if (nc == 2 && ks == 2) return loglik_pipe_entry<2, 2, false>();
    if (nc == 2 && ks == 4) return loglik_pipe_entry<2, 4, false>();
    return LoglikEntry{};
}

}  // namespace sps
