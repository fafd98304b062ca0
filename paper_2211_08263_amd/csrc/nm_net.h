// Solver-side interface of the learned warm start (implemented in nm_net.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define CHECK_NM(expr)                                                                                                 \
    do {                                                                                                               \
        int e_ = (expr);                                                                                               \
        if (e_ != 0) return e_;                                                                                        \
    } while (0)

struct nm_net;

namespace nm {

struct WarmArgs {
    int n1, n2, n3;
    long N;
    const double* u;       // u_n, SoA 3 x N
    const double* v;       // v_n
    const double* a;       // a_n
    const double* ut;      // Newmark predictor of the next step
    double dt, c2;         // dt and dt^2 (1/2 - beta)
    const uint16_t* phase; // grain id per voxel
    const float* matf;     // per phase: rho / rhobar, C_voigt[21] / Cbar_11
    double* red;           // >= 512 partial sums
    double* scale;         // one double: rms(u~ - u_n)
    uint16_t* feat;        // BF16 [N][32]
    uint16_t* l0mat;       // BF16 [N][16]: material share of layer 0 (with its bias)
    unsigned long long* l0mat_version; // network version l0mat was computed for (0: none)
    const double* inc = nullptr; // per-block sums of |u~ - u_n|^2 left by the corrector (null: summed here)
    int inc_nb = 0;              // number of those sums
    float* x0f = nullptr;        // warm_predict: FP32 copy of x0 as well (or null)
    uint16_t* sfeat = nullptr;   // warm_predict: unscaled BF16 state features [N][16]
    bool sfeat_ready = false;    // sfeat already holds them (written by the fused corrector)
};

int warm_features(const WarmArgs& a, hipStream_t s);
int warm_predict(nm_net* net, const WarmArgs& a, double* x0, hipStream_t s);
// target (u_next - u~)/s from the new acceleration: u_next - u~ = beta dt^2 a_next
int warm_target(const WarmArgs& a, const double* anext, double bdt2, float* target, hipStream_t s);
// Residual-norm training: y = scale * P net(feat) (FP64 SoA, Gamma voxels zero) ...
int warm_residual_forward(nm_net* net, const WarmArgs& a, const uint16_t* feat, double scale, const uint8_t* mask,
                          double* y, hipStream_t s);
// ... then, with dL/dpred = scale * gsoa (FP64 SoA), backward pass and one Adam step.
int warm_residual_backward(nm_net* net, const WarmArgs& a, const uint16_t* feat, const double* gsoa, double scale,
                           float lr, hipStream_t s);

} // namespace nm
