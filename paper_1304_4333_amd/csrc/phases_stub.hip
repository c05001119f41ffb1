// Temporary: the M phase entry point (kernels being written).
#include "sps_internal.h"
using namespace sps;
extern "C" int sps_mutate(sps_ctx*, double*, double*, double*, int32_t, int32_t, int64_t, double, int, int,
                          const double*, const double*, uint64_t, uint64_t, double*) { return SPS_ERR_ARG; }
