// Learned warm start (placeholder until the network kernels land).
#include "nm_warm.h"

namespace nm {

struct WarmNet {
    int dummy;
};

int warm_predict(WarmNet*, const double*, const double*, const double*, double*, double, hipStream_t) { return -1; }
void warm_destroy(WarmNet* net) { delete net; }

} // namespace nm
