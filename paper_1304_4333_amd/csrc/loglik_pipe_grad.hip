// loglik_pipe_grad.hip -- instantiations of the pipelined BF16x3 likelihood
// kernel (forward + adjoint), C = 2 outcomes, k > 32.
#include "loglik_pipe.h"

namespace sps {

LoglikEntry lookup_pipe_grad(int nc, int ks) {
    if (nc == 1 && ks == 2) return loglik_pipe_entry<1, 2, true>();
    if (nc == 1 && ks == 4) return loglik_pipe_entry<1, 4, true>();
    return LoglikEntry{};
}

}  // namespace sps
