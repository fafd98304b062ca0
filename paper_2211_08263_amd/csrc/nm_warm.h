// Learned warm start: a small periodic 3D convolutional network that predicts
// the next displacement from the current state (BF16 MFMA kernels).
#pragma once
#include <hip/hip_runtime.h>

namespace nm {

struct WarmNet;

// x0 = prediction of u_{n+1} from (u_n, v_n, a_n); Gamma entries are set by the caller afterwards.
int warm_predict(WarmNet* net, const double* u, const double* v, const double* a, double* x0, double dt,
                 hipStream_t s);
void warm_destroy(WarmNet* net);

} // namespace nm
