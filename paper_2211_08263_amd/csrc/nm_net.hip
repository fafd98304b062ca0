// Learned warm start: a small periodic 3D convolutional network (3x3x3
// kernels, 16 hidden channels, leaky ReLU) that predicts the correction to
// the Newmark predictor u~ = u + dt v + dt^2 (1/2 - beta) a:
//     x0 = u~ + s * net(features),  s = rms(u~ - u_n)
// features (channels-last BF16, 32 per voxel): u_n/s, dt v_n/s,
// dt^2 (1/2 - beta) a_n/s (the Newmark state, 9), rho/rhobar (1),
// C/Cbar_11 (21), 0 (1).
//
// Convolutions are implicit GEMMs on the BF16 matrix cores (MFMA 16x16x16,
// FP32 accumulation): a wave computes 16 consecutive voxels along x x 16
// output channels, looping over the 27 taps and the input-channel chunks.
// Operand layouts (per lane l, r = l % 16, g = l / 16):
//   A[row = r][k = 4g + i],  B[k = 4g + i][col = r],  D[row = 4g + i][col = r].
#include "../../include/newmark.h"
#include "nm_common.h"
#include <type_traits>
#include "nm_net.h"

#include <cmath>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

namespace nm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr float kLeak = 0.1f;
constexpr int kFeat = 32;   // padded feature channels
constexpr int kHid = 16;    // hidden channels (also the padded MFMA N)
constexpr int kOutC = 3;    // predicted displacement components
constexpr int kPredStride = 4;
constexpr int kState = 9;   // state feature channels (u, dt v, dt^2 (1/2 - beta) a)

__host__ __device__ inline uint16_t f2bf(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16); // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);                                   // round to nearest even
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

struct Grid {
    int n1, n2, n3;
    long N;
};

__device__ __forceinline__ long tap_voxel(int x, int y, int z, int t, const Grid& g)
{
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const int xx = (x + dx) & (g.n1 - 1), yy = (y + dy) & (g.n2 - 1), zz = (z + dz) & (g.n3 - 1);
    return ((long)zz * g.n2 + yy) * g.n1 + xx;
}

// ---------------------------------------------------------------------------
// Forward convolution: Y[v][co] = b[co] + sum_{tap, ci} W[tap][co][ci] X[v + d(tap)][ci]
//   X: BF16 [N][CINP], W: BF16 [27][16][CINP] (co padded to 16), bias FP32 [16].
// Epilogues: EPI_BF16_ACT  -> BF16 [N][16], leaky ReLU
//            EPI_F32       -> FP32 [N][ostride] (channels < cout), no activation
//            EPI_BF16_DACT -> BF16 [N][16] times leaky'(aux), aux BF16 [N][16] (backward data pass)
//            EPI_BF16_ACT_ADD -> BF16 [N][16], leaky ReLU of the sum with aux, BF16 [N][16]
//            EPI_BF16      -> BF16 [N][16], no activation
//
// A block owns a 16 (x) by TY (y) column of voxels over ZC consecutive z planes.
// It keeps three halo planes of the input ((TY + 2) x 18 voxels, all CINP
// channels, periodic wrap) in LDS and marches along z: while the waves compute
// one output plane from the three resident planes, the next input plane is
// already on its way into registers, and it replaces the oldest plane after a
// barrier.  Every input voxel is read from HBM about (1 + 2/TY)(1 + 2/16)(1 + 2/ZC)
// times instead of once per tap.  Wave w computes the 16-voxel rows y0 + w + 4 j
// (four independent MFMA accumulators); the weights stay in registers.
// LDS plane layout: [kc][row][col][16 channels] BF16, so the 64 lanes of one
// A-operand read cover 512 contiguous bytes.
// ---------------------------------------------------------------------------
enum { EPI_BF16_ACT = 0, EPI_F32 = 1, EPI_BF16_DACT = 2, EPI_BF16_ACT_ADD = 3, EPI_BF16 = 4 };

// EPI_BF16_ACT_ADD with scale set: the convolution output is multiplied by 1/scale[0]
// (0 if the scale is 0) before aux is added.
struct ConvExtra {
    const double* scale = nullptr;
};
constexpr int kTX = 16;            // x extent of a block tile
constexpr int kHX = kTX + 2;       // halo columns
constexpr int kMaxTY = 16;         // y extent of a block tile (rows of 16 voxels)
constexpr int kHR = kMaxTY + 2;    // halo rows

// Input plane z (wrapped) of a block's halo tile: global -> registers (16-byte chunks,
// chunk id = (row * 18 + col) * CINP/8 + q) and registers -> one LDS plane slot.
template <int CINP, int NCH>
__device__ __forceinline__ void conv_fetch(u32x4 (&buf)[NCH], const uint16_t* __restrict__ X, const Grid& g, int x0,
                                           int y0, int z, int nchunk)
{
    constexpr int QV = CINP / 8;
    const int zz = z & (g.n3 - 1);
#pragma unroll
    for (int k = 0; k < NCH; k++) {
        // chunks past the tile re-read chunk 0 (always in range) and are not stashed
        int id = threadIdx.x + 256 * k;
        id = id < nchunk ? id : 0;
        const int q = id % QV, vox = id / QV, col = vox % kHX, row = vox / kHX;
        const int gx = (x0 - 1 + col) & (g.n1 - 1), gy = (y0 - 1 + row) & (g.n2 - 1);
        buf[k] = *(const u32x4*)(X + (((long)zz * g.n2 + gy) * g.n1 + gx) * CINP + q * 8);
    }
}
template <int CINP, int NCH>
__device__ __forceinline__ void conv_stash(const u32x4 (&buf)[NCH], uint16_t* dst, int nchunk)
{
    constexpr int QV = CINP / 8;
#pragma unroll
    for (int k = 0; k < NCH; k++) {
        const int id = threadIdx.x + 256 * k;
        if (id < nchunk) {
            const int q = id % QV, vox = id / QV, col = vox % kHX, row = vox / kHX;
            *(u32x4*)(dst + (((q >> 1) * kHR + row) * kHX + col) * 16 + (q & 1) * 8) = buf[k];
        }
    }
}

// K steps of one input plane: CINP == 32 takes one in-plane tap (32 channels) per
// 16x16x32 MFMA; CINP == 16 takes two in-plane taps (16 channels each) per MFMA, lanes
// 0-31 of the A/B operands holding in-plane tap 2s and lanes 32-63 tap 2s + 1 (the
// tenth tap is padding with zero weights).
template <int CINP> struct ConvK {
    static constexpr int STEPS = CINP == 32 ? 9 : 5;
    // in-plane tap (dy, dx) = (t / 3, t % 3) whose channels lane group gq (0..3) supplies at step s
    static __device__ __forceinline__ int tap(int s, int gq) { return CINP == 32 ? s : 2 * s + (gq >> 1); }
};

// Input planes stream through LDS one at a time; each A fragment read from a plane
// feeds the three output planes it reaches (taps dz = 0, 1, 2 of outputs p, p - 1,
// p - 2 in plane-local indices), whose accumulators rotate over three register slots,
// so every A fragment is read from LDS once instead of three times.
template <int CINP, int EPI>
__global__ __launch_bounds__(256, CINP == 16 ? 3 : 2) void k_conv_fwd(const uint16_t* __restrict__ X, const uint16_t* __restrict__ W,
                                                  const float* __restrict__ bias, void* __restrict__ Y,
                                                  const void* __restrict__ aux, Grid g, int cout, int ostride,
                                                  int TY, int ZC, ConvExtra ex)
{
    constexpr int KC = CINP / 16;
    constexpr int PLANE = KC * kHR * kHX * 16;         // BF16 elements per plane slot
    constexpr int NCH = (kHR * kHX * (CINP / 8) + 255) / 256;
    constexpr int STEPS = ConvK<CINP>::STEPS;
    __shared__ __align__(16) uint16_t pl[2 * PLANE];
    __shared__ __align__(16) bf16x8 wl[3 * STEPS * 64]; // [dz][step][lane] B fragments
    __shared__ __align__(16) float stg[4][256];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, gq = lane >> 4;
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * TY, z0 = blockIdx.z * ZC;
    const int nchunk = (TY + 2) * kHX * (CINP / 8);

    // B fragment of lane (co, gq) at (dz, step): W[dz 9 + in-plane tap][co][ci .. ci + 7]
    for (int e = tid; e < 3 * STEPS * 64; e += 256) {
        const int l = e % 64, st = (e / 64) % STEPS, dz = e / (64 * STEPS), lg = l >> 4;
        const int t = ConvK<CINP>::tap(st, lg);
        const int ci = CINP == 32 ? 8 * lg : 8 * (lg & 1);
        bf16x8 w = {0, 0, 0, 0, 0, 0, 0, 0};
        if (t < 9) w = *(const bf16x8*)(W + ((long)((dz * 9 + t) * 16 + (l & 15)) * CINP + ci));
        wl[e] = w;
    }
    const float bcol = (bias && r < cout) ? bias[r] : 0.0f;
    float einv = 1.0f; // EPI_BF16_ACT_ADD: 1/s applied to the convolution output
    if constexpr (EPI == EPI_BF16_ACT_ADD) {
        if (ex.scale) einv = ex.scale[0] > 0.0 ? (float)(1.0 / ex.scale[0]) : 0.0f;
    }

    // A operand of this lane at step s: its in-plane tap's (dy, dx) and channel offset
    int aoff[STEPS];
#pragma unroll
    for (int st = 0; st < STEPS; st++) {
        int t = ConvK<CINP>::tap(st, gq);
        t = t < 9 ? t : 8; // padding tap: any finite input, zero weights
        const int dy = t / 3, dx = t % 3;
        const int kc = CINP == 32 ? (gq >> 1) : 0;
        aoff[st] = ((kc * kHR + dy) * kHX + dx + r) * 16 + 8 * (gq & 1);
    }
    int rowoff[4];
#pragma unroll
    for (int j = 0; j < 4; j++) rowoff[j] = min(wv + 4 * j, TY - 1) * (kHX * 16); // rows past TY: not written

    constexpr bool AUX = EPI == EPI_BF16_ACT_ADD || EPI == EPI_BF16_DACT;
    const int vv = lane >> 2, c0 = 4 * (lane & 3); // epilogue: lane owns voxel vv, channels c0 .. c0 + 3
    // the aux operand of output plane k (4 BF16 per row j), fetched ahead of the epilogue
    auto aux_fetch = [&](uint64_t (&ap)[4], int k) {
        const int z = z0 + k;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int ty = min(wv + 4 * j, TY - 1);
            const long v0 = ((long)z * g.n2 + (y0 + ty)) * g.n1 + x0;
            ap[j] = *(const uint64_t*)((const uint16_t*)aux + (v0 + vv) * kHid + c0);
        }
    };
    // output plane k (z0 + k) of this block from accumulator slot acc[k mod 3]
    auto epilogue = [&](const f32x4 (&ac)[4], int k, const uint64_t (&apre)[4]) {
        const int z = z0 + k;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int ty = wv + 4 * j;
            if (ty >= TY) continue;
            const long v0 = ((long)z * g.n2 + (y0 + ty)) * g.n1 + x0;
            if constexpr (EPI == EPI_F32) {
#pragma unroll
                for (int i = 0; i < 4; i++)
                    if (r < cout) ((float*)Y)[(v0 + 4 * gq + i) * ostride + r] = ac[j][i] + bcol;
            } else {
                // D (voxel 4 gq + i, channel r) -> staging -> lane L owns voxel L / 4, channels 4 (L % 4) .. + 3
#pragma unroll
                for (int i = 0; i < 4; i++) stg[wv][(4 * gq + i) * 16 + r] = ac[j][i] + bcol;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const float4 o4 = *(const float4*)&stg[wv][vv * 16 + c0];
                float o[4] = {o4.x, o4.y, o4.z, o4.w};
                if constexpr (EPI == EPI_BF16_ACT || EPI == EPI_BF16_ACT_ADD) {
                    if constexpr (EPI == EPI_BF16_ACT_ADD) {
                        // unscaled inputs: the convolution is linear, so 1/s applies to its output
#pragma unroll
                        for (int c = 0; c < 4; c++) o[c] *= einv;
                        const uint64_t ap = apre[j];
#pragma unroll
                        for (int c = 0; c < 4; c++) o[c] += bf2f((uint16_t)(ap >> (16 * c)));
                    }
#pragma unroll
                    for (int c = 0; c < 4; c++) o[c] = o[c] > 0.f ? o[c] : kLeak * o[c];
                } else if constexpr (EPI == EPI_BF16_DACT) {
                    const uint64_t ap = apre[j];
#pragma unroll
                    for (int c = 0; c < 4; c++) {
                        const float av = bf2f((uint16_t)(ap >> (16 * c)));
                        o[c] = av > 0.f ? o[c] : kLeak * o[c];
                    }
                }
                const uint64_t w = (uint64_t)f2bf(o[0]) | ((uint64_t)f2bf(o[1]) << 16) |
                                   ((uint64_t)f2bf(o[2]) << 32) | ((uint64_t)f2bf(o[3]) << 48);
                *(uint64_t*)((uint16_t*)Y + (v0 + vv) * kHid + c0) = w;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    };

    f32x4 acc[3][4];
#pragma unroll
    for (int q = 0; q < 3; q++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[q][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // plane-local input index p = 0 .. ZC + 1 is global plane z0 - 1 + p; LDS slot p % 2
    const int NP = ZC + 2;
    u32x4 bufA[NCH], bufB[NCH];
    conv_fetch<CINP, NCH>(bufA, X, g, x0, y0, z0 - 1, nchunk);
    conv_stash<CINP, NCH>(bufA, pl, nchunk);
    conv_fetch<CINP, NCH>(bufA, X, g, x0, y0, z0, nchunk);

    // SQ = p mod 3 (accumulator slot of output p); cur holds plane p + 1, nxt receives p + 2
    auto step = [&](int p, auto SQ, u32x4 (&cur)[NCH], u32x4 (&nxt)[NCH]) {
        constexpr int q0 = decltype(SQ)::value;       // output p     (dz = 0)
        constexpr int q1 = (q0 + 2) % 3;              // output p - 1 (dz = 1)
        constexpr int q2 = (q0 + 1) % 3;              // output p - 2 (dz = 2)
        __syncthreads(); // plane p is in slot p % 2; every wave is done with plane p - 1
        if (p + 1 < NP) conv_stash<CINP, NCH>(cur, pl + ((p + 1) & 1) * PLANE, nchunk);
        if (p + 2 < NP) conv_fetch<CINP, NCH>(nxt, X, g, x0, y0, z0 - 1 + p + 2, nchunk);
        const uint16_t* sb = pl + (p & 1) * PLANE;
        const bool o0 = p < ZC, o1 = p >= 1 && p - 1 < ZC, o2 = p >= 2;
        uint64_t apre[4] = {0, 0, 0, 0};
        if constexpr (AUX) {
            if (o2) aux_fetch(apre, p - 2);
        }
#pragma unroll
        for (int st = 0; st < STEPS; st++) {
            const bf16x8 b0 = wl[(0 * STEPS + st) * 64 + lane];
            const bf16x8 b1 = wl[(1 * STEPS + st) * 64 + lane];
            const bf16x8 b2 = wl[(2 * STEPS + st) * 64 + lane];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const bf16x8 a = *(const bf16x8*)(sb + aoff[st] + rowoff[j]);
                if (o0) acc[q0][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc[q0][j], 0, 0, 0);
                if (o1) acc[q1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc[q1][j], 0, 0, 0);
                if (o2) acc[q2][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b2, acc[q2][j], 0, 0, 0);
            }
        }
        // output p - 2 has all three contributions
        if (o2) {
            epilogue(acc[q2], p - 2, apre);
#pragma unroll
            for (int j = 0; j < 4; j++) acc[q2][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    };
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    using S2 = std::integral_constant<int, 2>;
    for (int p = 0; p < NP; p += 6) {
        step(p, S0{}, bufA, bufB);
        if (p + 1 < NP) step(p + 1, S1{}, bufB, bufA);
        if (p + 2 < NP) step(p + 2, S2{}, bufA, bufB);
        if (p + 3 < NP) step(p + 3, S0{}, bufB, bufA);
        if (p + 4 < NP) step(p + 4, S1{}, bufA, bufB);
        if (p + 5 < NP) step(p + 5, S2{}, bufB, bufA);
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[co][ci][tap] = sum_v dZ[v][co] X[v + d(tap)][ci]  (MFMA with
// K = voxels), bias gradient db[co] = sum_v dZ[v][co].  Each wave writes its
// partial sums; k_reduce_partials adds them in a fixed order.
//   partial layout per wave: [27][KC][64 lanes][4] then [64 lanes] (bias)
// A tile is 16 consecutive voxels of one x row.  With 32 input channels, for each (dz, dy)
// the wave stages the 18 source voxels x0 - 1 .. x0 + 16 of that row (every channel) in its
// own LDS slot with 16-byte loads, and the three dx taps take their operands from there
// (1.61 -> 1.18 ms at 128^3 against per-lane 2-byte gathers); 16 input channels keep the
// gathers.
// ---------------------------------------------------------------------------
template <int CINP>
__global__ __launch_bounds__(256) void k_conv_bwdw(const uint16_t* __restrict__ X, const uint16_t* __restrict__ DZ,
                                                   float* __restrict__ partial, Grid g, long tiles_per_wave)
{
    constexpr int KC = CINP / 16;
    constexpr long PW = 27L * KC * 256 + 64;
    constexpr int CPV = CINP / 8;          // 16-byte chunks per voxel
    constexpr int ROWCH = 18 * CPV;        // chunks of one staged row
    __shared__ u32x4 rows[4][ROWCH];       // one staged row per wave of the block
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const long wave = (long)blockIdx.x * (blockDim.x / 64) + wv;
    const int r = lane & 15, gq = lane >> 4;
    const long ntiles = g.N / 16;
    // waves past the last tile range own no partial slot
    if (wave * tiles_per_wave >= ntiles) return;
    const uint16_t* rowl = (const uint16_t*)rows[wv];
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    f32x4 acc[27][KC];
#pragma unroll
    for (int t = 0; t < 27; t++)
#pragma unroll
        for (int kc = 0; kc < KC; kc++) acc[t][kc] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    const long t0 = wave * tiles_per_wave;
    const long t1 = t0 + tiles_per_wave < ntiles ? t0 + tiles_per_wave : ntiles;
    for (long tile = t0; tile < t1; tile++) {
        const long v0 = tile * 16;
        const int x0 = (int)(v0 & (g.n1 - 1));
        const long yz = v0 / g.n1;
        const int y = (int)(yz % g.n2), z = (int)(yz / g.n2);
        bf16x4 b;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint16_t h = DZ[(v0 + 4 * gq + i) * kHid + r];
            b[i] = (short)h;
            bsum += bf2f(h);
        }
        if constexpr (CINP == 16) {
            // 16 channels: the per-lane gathers from the caches beat the staging, whose nine
            // rounds per tile each wait for their loads (0.55 against 0.78 ms at 128^3)
#pragma unroll
            for (int t = 0; t < 27; t++) {
                long vs[4];
#pragma unroll
                for (int i = 0; i < 4; i++) vs[i] = tap_voxel(x0 + 4 * gq + i, y, z, t, g);
                bf16x4 a;
#pragma unroll
                for (int i = 0; i < 4; i++) a[i] = (short)X[vs[i] * CINP + r];
                acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t][0], 0, 0, 0);
            }
            continue;
        }
#pragma unroll
        for (int dzy = 0; dzy < 9; dzy++) {
            const int zz = (z + dzy / 3 - 1) & (g.n3 - 1), yy = (y + dzy % 3 - 1) & (g.n2 - 1);
            const long rbase = ((long)zz * g.n2 + yy) * g.n1;
            wave_sync(); // every lane is done with the previous row
            for (int c = lane; c < ROWCH; c += 64) {
                const int j = c / CPV, q = c % CPV;
                const int xx = (x0 - 1 + j) & (g.n1 - 1);
                rows[wv][c] = *(const u32x4*)(X + (rbase + xx) * CINP + q * 8);
            }
            wave_sync();
#pragma unroll
            for (int dx = 0; dx < 3; dx++) {
                // tap (dz, dy, dx) in tap_voxel's order; element i of this lane is voxel
                // x0 + 4 gq + i + dx - 1, staged at j = 4 gq + i + dx
                const int t = dzy * 3 + dx;
#pragma unroll
                for (int kc = 0; kc < KC; kc++) {
                    bf16x4 a;
#pragma unroll
                    for (int i = 0; i < 4; i++) a[i] = (short)rowl[(4 * gq + i + dx) * CINP + kc * 16 + r];
                    acc[t][kc] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t][kc], 0, 0, 0);
                }
            }
        }
    }
    float* out = partial + wave * PW;
#pragma unroll
    for (int t = 0; t < 27; t++)
#pragma unroll
        for (int kc = 0; kc < KC; kc++)
#pragma unroll
            for (int i = 0; i < 4; i++) out[((long)(t * KC + kc) * 64 + lane) * 4 + i] = acc[t][kc][i];
    out[27L * KC * 256 + lane] = bsum;
}

// Sum the per-wave partials (fixed order) and scatter into dW[co][ci][tap], db[co].
// D element (lane l, reg i) of chunk kc = [row ci = kc*16 + 4*(l/16) + i][col co = l % 16].
template <int CINP>
__global__ void k_reduce_bwdw(const float* __restrict__ partial, int nwaves, float* __restrict__ dW,
                              float* __restrict__ db, int cin, int cout)
{
    constexpr int KC = CINP / 16;
    constexpr long PW = 27L * KC * 256 + 64;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 27L * KC * 256) {
        float s = 0.f;
        for (int w = 0; w < nwaves; w++) s += partial[w * PW + e];
        const int i = (int)(e % 4), lane = (int)((e / 4) % 64), tk = (int)(e / 256);
        const int t = tk / KC, kc = tk % KC;
        const int ci = kc * 16 + 4 * (lane / 16) + i, co = lane % 16;
        if (ci < cin && co < cout) dW[((long)co * cin + ci) * 27 + t] = s;
    } else if (e < 27L * KC * 256 + 16) {
        const int co = (int)(e - 27L * KC * 256);
        float s = 0.f;
        for (int w = 0; w < nwaves; w++)
            for (int q = 0; q < 4; q++) s += partial[w * PW + 27L * KC * 256 + co + 16 * q];
        if (co < cout) db[co] = s;
    }
}

// ---------------------------------------------------------------------------
// Loss: L = mean over voxels and components of (pred - target)^2;
// dZ = dL/dpred as BF16 [N][16] (channels >= 3 zero).  Per-block partial sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ pred, const float* __restrict__ target,
                                              uint16_t* __restrict__ dz, long N, double* partials)
{
    __shared__ double sh[4];
    double acc = 0.0;
    const float sc = 2.0f / (float)(3.0 * (double)N);
    for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += (long)gridDim.x * blockDim.x) {
        uint16_t o[kHid];
#pragma unroll
        for (int c = 0; c < kHid; c++) o[c] = 0;
#pragma unroll
        for (int c = 0; c < kOutC; c++) {
            const float d = pred[v * kPredStride + c] - target[v * kPredStride + c];
            acc += (double)d * d;
            o[c] = f2bf(sc * d);
        }
#pragma unroll
        for (int c = 0; c < kHid; c++) dz[v * kHid + c] = o[c];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (sh[0] + sh[1] + sh[2] + sh[3]) / (3.0 * (double)N);
}

// ---------------------------------------------------------------------------
// Adam on the FP32 master parameters, then BF16 packing of the weights.
// ---------------------------------------------------------------------------
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Forward layout Wf[tap][16][cinp] (co padded) and backward-data layout
// Wb[tap'][16 (ci)][16 (co)] = W[co][ci][26 - tap'] (flipped taps, transposed).
__global__ void k_pack(const float* __restrict__ W, int cin, int cout, int cinp, uint16_t* __restrict__ Wf,
                       uint16_t* __restrict__ Wb)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = 27 * 16 * cinp;
    if (e < nf) {
        const int ci = e % cinp, co = (e / cinp) % 16, t = e / (16 * cinp);
        Wf[e] = (ci < cin && co < cout) ? f2bf(W[((long)co * cin + ci) * 27 + t]) : (uint16_t)0;
    }
    if (Wb && e < 27 * 256) {
        const int co = e % 16, ci = (e / 16) % 16, t = e / 256;
        Wb[e] = (ci < cin && co < cout) ? f2bf(W[((long)co * cin + ci) * 27 + (26 - t)]) : (uint16_t)0;
    }
}

// Layer 0 restricted to the state channels (ci < 9) in the 16-channel forward layout
// Wf0s[tap][16 (co)][16 (ci)]; W0 is [16][31][27].
__global__ void k_pack_state(const float* __restrict__ W0, uint16_t* __restrict__ Wf0s)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 27 * 256) return;
    const int ci = e % 16, co = (e / 16) % 16, t = e / 256;
    Wf0s[e] = ci < kState ? f2bf(W0[((long)co * 31 + ci) * 27 + t]) : (uint16_t)0;
}

// ---------------------------------------------------------------------------
// Features and prediction
// ---------------------------------------------------------------------------
// partial sums of |u~ - u|^2 (u~ = predictor), for the scale s
__global__ __launch_bounds__(256) void k_incr_norm(const double* __restrict__ ut, const double* __restrict__ u, long n,
                                                   double* partials)
{
    __shared__ double sh[4];
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double d = ut[i] - u[i];
        acc += d * d;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// scale = sqrt(sum of the partials / count); one wavefront, fixed summation order
__global__ __launch_bounds__(64) void k_sum_scale(const double* __restrict__ partials, int n, long count,
                                                  double* scale)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) s += partials[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    // s = 0 before anything moves: features are zero and the correction vanishes
    if (threadIdx.x == 0) scale[0] = sqrt(s / (double)count);
}

__global__ __launch_bounds__(256) void k_features(const double* __restrict__ u, const double* __restrict__ v,
                                                  const double* __restrict__ a, double dt, double c2,
                                                  const uint16_t* __restrict__ phase, const float* __restrict__ matf,
                                                  long N, const double* __restrict__ scale, uint16_t* __restrict__ X)
{
    const double inv = scale[0] > 0.0 ? 1.0 / scale[0] : 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
        uint16_t f[kFeat];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            f[c] = f2bf((float)(u[c * N + i] * inv));
            f[3 + c] = f2bf((float)(dt * v[c * N + i] * inv));
            f[6 + c] = f2bf((float)(c2 * a[c * N + i] * inv));
        }
        const float* mf = matf + 22 * (long)phase[i];
#pragma unroll
        for (int c = 0; c < 22; c++) f[9 + c] = f2bf(mf[c]);
        f[31] = 0;
#pragma unroll
        for (int c = 0; c < kFeat; c += 4) {
            uint64_t w = (uint64_t)f[c] | ((uint64_t)f[c + 1] << 16) | ((uint64_t)f[c + 2] << 32) |
                         ((uint64_t)f[c + 3] << 48);
            *(uint64_t*)(X + i * kFeat + c) = w;
        }
    }
}

// Inference features, state part only: BF16 [N][16], channels 0..8 as in k_features, rest 0.
__global__ __launch_bounds__(256) void k_features_state(const double* __restrict__ u, const double* __restrict__ v,
                                                        const double* __restrict__ a, double dt, double c2, long N,
                                                        const double* __restrict__ scale, uint16_t* __restrict__ X)
{
    // scale null: unscaled features (the solver's first layer applies 1/s itself)
    const double inv = scale ? (scale[0] > 0.0 ? 1.0 / scale[0] : 0.0) : 1.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
        uint16_t f[16];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            f[c] = f2bf((float)(u[c * N + i] * inv));
            f[3 + c] = f2bf((float)(dt * v[c * N + i] * inv));
            f[6 + c] = f2bf((float)(c2 * a[c * N + i] * inv));
        }
#pragma unroll
        for (int c = kState; c < 16; c++) f[c] = 0;
#pragma unroll
        for (int c = 0; c < 16; c += 4) {
            const uint64_t w = (uint64_t)f[c] | ((uint64_t)f[c + 1] << 16) | ((uint64_t)f[c + 2] << 32) |
                               ((uint64_t)f[c + 3] << 48);
            *(uint64_t*)(X + i * 16 + c) = w;
        }
    }
}

// Material part of the features: BF16 [N][32] with the state channels zero.
__global__ __launch_bounds__(256) void k_features_material(const uint16_t* __restrict__ phase,
                                                           const float* __restrict__ matf, long N,
                                                           uint16_t* __restrict__ X)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
        uint16_t f[kFeat];
#pragma unroll
        for (int c = 0; c < kState; c++) f[c] = 0;
        const float* mf = matf + 22 * (long)phase[i];
#pragma unroll
        for (int c = 0; c < 22; c++) f[kState + c] = f2bf(mf[c]);
        f[31] = 0;
#pragma unroll
        for (int c = 0; c < kFeat; c += 4) {
            const uint64_t w = (uint64_t)f[c] | ((uint64_t)f[c + 1] << 16) | ((uint64_t)f[c + 2] << 32) |
                               ((uint64_t)f[c + 3] << 48);
            *(uint64_t*)(X + i * kFeat + c) = w;
        }
    }
}

// x0 = u~ + s * pred (SoA FP64 out; x0f, if given, receives the FP32 copy)
__global__ __launch_bounds__(256) void k_predict(const double* __restrict__ ut, const float* __restrict__ pred,
                                                 const double* __restrict__ scale, double* __restrict__ x0,
                                                 float* __restrict__ x0f, long N)
{
    const double s = scale[0];
    for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += (long)gridDim.x * blockDim.x)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const double x = ut[c * N + v] + s * (double)pred[v * kPredStride + c];
            x0[c * N + v] = x;
            if (x0f) x0f[c * N + v] = (float)x;
        }
}

// target = (u_next - u~) / s = beta dt^2 a_next / s  (the corrector's definition of
// a_next), as FP32 [N][4]
__global__ __launch_bounds__(256) void k_target(const double* __restrict__ anext, double bdt2,
                                                const double* __restrict__ scale, float* __restrict__ target, long N)
{
    const double inv = scale[0] > 0.0 ? bdt2 / scale[0] : 0.0;
    for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += (long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < 3; c++) target[v * kPredStride + c] = (float)(anext[c * N + v] * inv);
        target[v * kPredStride + 3] = 0.f;
    }
}

// y = s * P pred as FP64 SoA 3 x N (Gamma voxels zero)
__global__ __launch_bounds__(256) void k_pred_soa(const float* __restrict__ pred, double s,
                                                  const uint8_t* __restrict__ mask, long N, double* __restrict__ y)
{
    for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += (long)gridDim.x * blockDim.x) {
        const bool fixed = mask && mask[v];
#pragma unroll
        for (int c = 0; c < 3; c++) y[c * N + v] = fixed ? 0.0 : s * (double)pred[v * kPredStride + c];
    }
}

// dz (BF16 [N][16]) = scale * g (FP64 SoA 3 x N), channels >= 3 zero
__global__ __launch_bounds__(256) void k_dz_soa(const double* __restrict__ g, double scale, long N,
                                                uint16_t* __restrict__ dz)
{
    for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += (long)gridDim.x * blockDim.x) {
        uint16_t o[kHid];
#pragma unroll
        for (int c = 0; c < kHid; c++) o[c] = 0;
#pragma unroll
        for (int c = 0; c < kOutC; c++) o[c] = f2bf((float)(scale * g[c * N + v]));
#pragma unroll
        for (int c = 0; c < kHid; c += 4) {
            const uint64_t w = (uint64_t)o[c] | ((uint64_t)o[c + 1] << 16) | ((uint64_t)o[c + 2] << 32) |
                               ((uint64_t)o[c + 3] << 48);
            *(uint64_t*)(dz + v * kHid + c) = w;
        }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int launch_conv(int cinp, int epi, const uint16_t* X, const uint16_t* W, const float* bias, void* Y,
                       const void* aux, const Grid& g, int cout, int ostride, hipStream_t s,
                       const ConvExtra& ex = ConvExtra{})
{
    // tiles: 16 x TY x ZC voxels per block (grid dimensions are powers of two, n1 >= 16)
    const int TY = g.n2 < kMaxTY ? g.n2 : kMaxTY;
    const int ZC = g.n3 < 16 ? g.n3 : 16;
    const dim3 grid(g.n1 / kTX, g.n2 / TY, g.n3 / ZC);
    if (g.n1 % kTX) return -1;
#define NM_CONV_LAUNCH(CI, EP)                                                                                         \
    hipLaunchKernelGGL((k_conv_fwd<CI, EP>), grid, dim3(256), 0, s, X, W, bias, Y, aux, g, cout, ostride, TY, ZC, ex)
    if (cinp == 32 && epi == EPI_BF16_ACT) NM_CONV_LAUNCH(32, EPI_BF16_ACT);
    else if (cinp == 32 && epi == EPI_F32) NM_CONV_LAUNCH(32, EPI_F32);
    else if (cinp == 16 && epi == EPI_BF16_ACT) NM_CONV_LAUNCH(16, EPI_BF16_ACT);
    else if (cinp == 16 && epi == EPI_F32) NM_CONV_LAUNCH(16, EPI_F32);
    else if (cinp == 16 && epi == EPI_BF16_DACT) NM_CONV_LAUNCH(16, EPI_BF16_DACT);
    else if (cinp == 16 && epi == EPI_BF16_ACT_ADD) NM_CONV_LAUNCH(16, EPI_BF16_ACT_ADD);
    else if (cinp == 32 && epi == EPI_BF16) NM_CONV_LAUNCH(32, EPI_BF16);
    else return -1;
#undef NM_CONV_LAUNCH
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Waves of the weight-gradient pass (each owns a partial-sum slot of bwdw_slot_floats(cinp)).
constexpr long kBwdwWaves = 1024;
static long bwdw_waves(long ntiles, long cap = kBwdwWaves) { return ntiles < cap ? ntiles : cap; }
static constexpr long bwdw_slot_floats(int cinp) { return 27L * (cinp / 16) * 256 + 64; }

static int launch_bwdw(int cinp, const uint16_t* X, const uint16_t* DZ, float* partial, float* dW, float* db, int cin,
                       int cout, const Grid& g, hipStream_t s, long wave_cap = kBwdwWaves)
{
    const long ntiles = g.N / 16;
    long waves = bwdw_waves(ntiles, wave_cap);
    const long tpw = (ntiles + waves - 1) / waves;
    waves = (ntiles + tpw - 1) / tpw;
    const int blocks = (int)((waves + 3) / 4);
    const long nout = 27L * (cinp / 16) * 256 + 16;
    if (cinp == 32) {
        hipLaunchKernelGGL((k_conv_bwdw<32>), dim3(blocks), dim3(256), 0, s, X, DZ, partial, g, tpw);
        hipLaunchKernelGGL((k_reduce_bwdw<32>), dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, partial,
                           (int)waves, dW, db, cin, cout);
    } else {
        hipLaunchKernelGGL((k_conv_bwdw<16>), dim3(blocks), dim3(256), 0, s, X, DZ, partial, g, tpw);
        hipLaunchKernelGGL((k_reduce_bwdw<16>), dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, partial,
                           (int)waves, dW, db, cin, cout);
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

} // namespace nm

using namespace nm;

// Network: layer l has cin_l -> cout_l, cinp_l padded input channels.
struct nm_net {
    int L = 4;
    int cin[4] = {31, 16, 16, 16}, cout[4] = {16, 16, 16, 3}, cinp[4] = {32, 16, 16, 16};
    long off[5] = {0, 0, 0, 0, 0}; // parameter offsets: W then b per layer
    long nparam = 0;
    float *p = nullptr, *gr = nullptr, *m = nullptr, *v = nullptr; // device FP32
    uint16_t* wf[4] = {};                                         // forward BF16
    uint16_t* wb[4] = {};                                         // backward-data BF16
    uint16_t* wf0s = nullptr; // layer 0 restricted to the 9 state channels, 16-channel layout
    unsigned long long version = 0; // bumped whenever the weights change
    long step = 0;
    // workspace (grown on demand)
    long capN = 0;
    uint16_t* act[4] = {}; // act[0] unused (features are the input), act[1..3] hidden
    uint16_t *dz0 = nullptr, *dz1 = nullptr;
    float* pred = nullptr;
    float* partial = nullptr;
    long cap_partial = 0;
    double* red = nullptr;
    double* hred = nullptr;
    std::vector<void*> ws_allocs;
};

static long layer_w(const nm_net* n, int l) { return (long)n->cout[l] * n->cin[l] * 27; }

static int net_alloc(void** p, size_t bytes, std::vector<void*>* list)
{
    if (hipMalloc(p, bytes) != hipSuccess) return NM_ENOMEM;
    if (list) list->push_back(*p);
    return NM_OK;
}

static int net_pack(nm_net* n, hipStream_t s)
{
    for (int l = 0; l < n->L; l++) {
        const int nf = 27 * 16 * n->cinp[l];
        const int tot = nf > 27 * 256 ? nf : 27 * 256;
        hipLaunchKernelGGL(k_pack, dim3((tot + 255) / 256), dim3(256), 0, s, n->p + n->off[l], n->cin[l],
                           n->cout[l], n->cinp[l], n->wf[l], l > 0 ? n->wb[l] : nullptr);
    }
    hipLaunchKernelGGL(k_pack_state, dim3(27), dim3(256), 0, s, n->p + n->off[0], n->wf0s);
    n->version++;
    return hipGetLastError() == hipSuccess ? NM_OK : NM_EHIP;
}

static int net_workspace(nm_net* n, long N)
{
    if (N <= n->capN) return NM_OK;
    for (void* q : n->ws_allocs) (void)hipFree(q);
    n->ws_allocs.clear();
    n->capN = 0;
    for (int l = 1; l < 4; l++) CHECK_NM(net_alloc((void**)&n->act[l], N * kHid * 2, &n->ws_allocs));
    CHECK_NM(net_alloc((void**)&n->dz0, N * kHid * 2, &n->ws_allocs));
    CHECK_NM(net_alloc((void**)&n->dz1, N * kHid * 2, &n->ws_allocs));
    CHECK_NM(net_alloc((void**)&n->pred, N * kPredStride * 4, &n->ws_allocs));
    const long waves = bwdw_waves(N / 16);
    CHECK_NM(net_alloc((void**)&n->partial, waves * (27L * 2 * 256 + 64) * 4, &n->ws_allocs));
    CHECK_NM(net_alloc((void**)&n->red, 4096 * sizeof(double), &n->ws_allocs));
    n->capN = N;
    return NM_OK;
}

extern "C" {

int nm_net_create(unsigned long long seed, nm_net** out)
{
    if (!out) return NM_EINVAL;
    nm_net* n = new nm_net();
    long o = 0;
    for (int l = 0; l < n->L; l++) {
        n->off[l] = o;
        o += layer_w(n, l) + n->cout[l];
    }
    n->off[4] = o;
    n->nparam = o;
    std::vector<float> h(o, 0.0f);
    std::mt19937_64 rng(seed);
    for (int l = 0; l < n->L; l++) {
        // He-style uniform init scaled for the leaky ReLU; the last layer starts small
        const float lim = (l == n->L - 1 ? 0.1f : 1.0f) * std::sqrt(6.0f / (27.0f * n->cin[l]));
        std::uniform_real_distribution<float> U(-lim, lim);
        for (long i = 0; i < layer_w(n, l); i++) h[n->off[l] + i] = U(rng);
    }
    int st = NM_OK;
    st |= net_alloc((void**)&n->p, o * 4, nullptr);
    st |= net_alloc((void**)&n->gr, o * 4, nullptr);
    st |= net_alloc((void**)&n->m, o * 4, nullptr);
    st |= net_alloc((void**)&n->v, o * 4, nullptr);
    for (int l = 0; l < n->L; l++) {
        st |= net_alloc((void**)&n->wf[l], 27 * 16 * n->cinp[l] * 2, nullptr);
        st |= net_alloc((void**)&n->wb[l], 27 * 256 * 2, nullptr);
    }
    st |= net_alloc((void**)&n->wf0s, 27 * 256 * 2, nullptr);
    if (st != NM_OK || hipHostMalloc((void**)&n->hred, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        nm_net_destroy(n);
        return NM_ENOMEM;
    }
    if (hipMemcpy(n->p, h.data(), o * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n->m, 0, o * 4) != hipSuccess || hipMemset(n->v, 0, o * 4) != hipSuccess ||
        hipMemset(n->gr, 0, o * 4) != hipSuccess || net_pack(n, nullptr) != NM_OK ||
        hipDeviceSynchronize() != hipSuccess) {
        nm_net_destroy(n);
        return NM_EHIP;
    }
    *out = n;
    return NM_OK;
}

void nm_net_destroy(nm_net* n)
{
    if (!n) return;
    (void)hipDeviceSynchronize();
    void* ptrs[] = {n->p, n->gr, n->m, n->v};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    for (int l = 0; l < 4; l++) {
        if (n->wf[l]) (void)hipFree(n->wf[l]);
        if (n->wb[l]) (void)hipFree(n->wb[l]);
    }
    if (n->wf0s) (void)hipFree(n->wf0s);
    for (void* q : n->ws_allocs) (void)hipFree(q);
    if (n->hred) (void)hipHostFree(n->hred);
    delete n;
}

long nm_net_num_params(const nm_net* n) { return n ? n->nparam : 0; }

int nm_net_get_params(const nm_net* n, float* w)
{
    if (!n || !w) return NM_EINVAL;
    return hipMemcpy(w, n->p, n->nparam * 4, hipMemcpyDeviceToHost) == hipSuccess ? NM_OK : NM_EHIP;
}

int nm_net_set_params(nm_net* n, const float* w)
{
    if (!n || !w) return NM_EINVAL;
    if (hipMemcpy(n->p, w, n->nparam * 4, hipMemcpyHostToDevice) != hipSuccess) return NM_EHIP;
    if (hipMemset(n->m, 0, n->nparam * 4) != hipSuccess || hipMemset(n->v, 0, n->nparam * 4) != hipSuccess)
        return NM_EHIP;
    n->step = 0;
    if (net_pack(n, nullptr) != NM_OK) return NM_EHIP;
    return hipDeviceSynchronize() == hipSuccess ? NM_OK : NM_EHIP;
}

static int check_grid(const int* n3)
{
    for (int i = 0; i < 3; i++)
        if (n3[i] < 1 || n3[i] > 1024 || (n3[i] & (n3[i] - 1))) return NM_EUNSUPPORTED;
    if (n3[0] < 16) return NM_EUNSUPPORTED;
    return NM_OK;
}

// Forward pass: feat BF16 [N][32] -> pred FP32 [N][4] (device).  Uses the
// network's workspace; pred_out may be NULL (then the internal buffer is kept).
static int net_forward(nm_net* n, const Grid& g, const uint16_t* feat, hipStream_t s)
{
    CHECK_NM(net_workspace(n, g.N));
    const uint16_t* in = feat;
    for (int l = 0; l < n->L; l++) {
        const float* b = n->p + n->off[l] + layer_w(n, l);
        int e;
        if (l < n->L - 1) e = launch_conv(n->cinp[l], EPI_BF16_ACT, in, n->wf[l], b, n->act[l + 1], nullptr, g, 16, 16, s);
        else e = launch_conv(n->cinp[l], EPI_F32, in, n->wf[l], b, n->pred, nullptr, g, n->cout[l], kPredStride, s);
        if (e) return e == -1 ? NM_EUNSUPPORTED : NM_EHIP;
        in = n->act[l + 1];
    }
    return NM_OK;
}

// Backward pass from dL/dpred already in dz0 (BF16 [N][16], channels >= 3 zero):
// parameter gradients into gr.  Needs the activations of a forward pass on feat.
static int net_backward(nm_net* n, const Grid& g, const uint16_t* feat, hipStream_t s)
{
    uint16_t *dz = n->dz0, *dznext = n->dz1;
    for (int l = n->L - 1; l >= 0; l--) {
        const uint16_t* in = l == 0 ? feat : n->act[l];
        float* gW = n->gr + n->off[l];
        if (launch_bwdw(n->cinp[l], in, dz, n->partial, gW, gW + layer_w(n, l), n->cin[l], n->cout[l], g, s))
            return NM_EHIP;
        if (l > 0) {
            // dZ_{l-1} = (W_l^T * dZ_l) . leaky'(A_{l-1}),  A_{l-1} = act[l]
            if (launch_conv(16, EPI_BF16_DACT, dz, n->wb[l], nullptr, dznext, n->act[l], g, 16, 16, s))
                return NM_EHIP;
            std::swap(dz, dznext);
        }
    }
    return NM_OK;
}

// Adam step on the master parameters and BF16 repack.
static int net_adam(nm_net* n, float lr, hipStream_t s)
{
    n->step++;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, (float)n->step), c2 = 1.f - std::pow(b2, (float)n->step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n->nparam + 255) / 256)), dim3(256), 0, s, n->p, n->gr, n->m, n->v,
                       n->nparam, lr, b1, b2, eps, c1, c2);
    return net_pack(n, s);
}

int nm_net_forward(nm_net* n, void* stream, const int* grid, const void* feat_dev, void* pred_dev)
{
    if (!n || !grid || !feat_dev || !pred_dev) return NM_EINVAL;
    CHECK_NM(check_grid(grid));
    Grid g{grid[0], grid[1], grid[2], (long)grid[0] * grid[1] * grid[2]};
    hipStream_t s = (hipStream_t)stream;
    CHECK_NM(net_forward(n, g, (const uint16_t*)feat_dev, s));
    if (hipMemcpyAsync(pred_dev, n->pred, g.N * kPredStride * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return NM_EHIP;
    return hipStreamSynchronize(s) == hipSuccess ? NM_OK : NM_EHIP;
}

int nm_net_train_step(nm_net* n, void* stream, const int* grid, const void* feat_dev, const void* target_dev,
                      float lr, float* loss)
{
    if (!n || !grid || !feat_dev || !target_dev || !(lr > 0)) return NM_EINVAL;
    CHECK_NM(check_grid(grid));
    Grid g{grid[0], grid[1], grid[2], (long)grid[0] * grid[1] * grid[2]};
    hipStream_t s = (hipStream_t)stream;
    const uint16_t* feat = (const uint16_t*)feat_dev;
    CHECK_NM(net_forward(n, g, feat, s));
    // loss and dL/dpred
    const int lb = 512;
    hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, s, n->pred, (const float*)target_dev, n->dz0, g.N, n->red);
    CHECK_NM(net_backward(n, g, feat, s));
    if (net_adam(n, lr, s) != NM_OK) return NM_EHIP;
    if (loss) {
        std::vector<double> part(lb);
        if (hipMemcpyAsync(part.data(), n->red, lb * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
            return NM_EHIP;
        if (hipStreamSynchronize(s) != hipSuccess) return NM_EHIP;
        double t = 0;
        for (int i = 0; i < lb; i++) t += part[i];
        *loss = (float)t;
    } else if (hipStreamSynchronize(s) != hipSuccess) {
        return NM_EHIP;
    }
    return hipGetLastError() == hipSuccess ? NM_OK : NM_EHIP;
}

int nm_net_gradients(nm_net* n, void* stream, const int* grid, const void* feat_dev, const void* target_dev,
                     float* grad_host, float* loss)
{
    // Same as one training step without the parameter update.
    if (!n || !grid || !feat_dev || !target_dev || !grad_host) return NM_EINVAL;
    CHECK_NM(check_grid(grid));
    Grid g{grid[0], grid[1], grid[2], (long)grid[0] * grid[1] * grid[2]};
    hipStream_t s = (hipStream_t)stream;
    const uint16_t* feat = (const uint16_t*)feat_dev;
    CHECK_NM(net_forward(n, g, feat, s));
    const int lb = 512;
    hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, s, n->pred, (const float*)target_dev, n->dz0, g.N, n->red);
    CHECK_NM(net_backward(n, g, feat, s));
    std::vector<double> part(lb);
    if (hipMemcpyAsync(part.data(), n->red, lb * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(grad_host, n->gr, n->nparam * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return NM_EHIP;
    if (loss) {
        double t = 0;
        for (int i = 0; i < lb; i++) t += part[i];
        *loss = (float)t;
    }
    return NM_OK;
}

// Single-layer kernels on caller buffers (used to check each kernel against the oracle).
// Device buffers of one call: FP32 weights and bias, their packed BF16 forms, and for the
// weight gradient the per-wave partial sums and the reduced gradients.
struct ConvBufs {
    float *wd = nullptr, *bd = nullptr, *part = nullptr, *dw = nullptr, *db = nullptr;
    uint16_t *wf = nullptr, *wb = nullptr;
};

__global__ void k_zero_f32(float* __restrict__ x, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.f;
}

static int conv3d_check(const int* grid, int cinp, int cin, int cout)
{
    if (!grid || (cinp != 16 && cinp != 32) || cin > cinp || cout > 16 || cin < 1 || cout < 1) return NM_EINVAL;
    return check_grid(grid);
}

static int conv3d_run(hipStream_t s, int mode, const Grid& g, int cinp, int cin, int cout, const void* x_dev,
                      const void* w_fp32_host, const float* bias_host, const void* dy_dev, void* out_dev,
                      float* dw_host, float* db_host, const ConvBufs& b, long wave_cap)
{
    const long nw = (long)cout * cin * 27;
    if (w_fp32_host && hipMemcpyAsync(b.wd, w_fp32_host, nw * 4, hipMemcpyHostToDevice, s) != hipSuccess)
        return NM_EHIP;
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, b.bd, 16);
    if (bias_host && hipMemcpyAsync(b.bd, bias_host, cout * 4, hipMemcpyHostToDevice, s) != hipSuccess) return NM_EHIP;
    {
        const int tot = 27 * 16 * cinp > 27 * 256 ? 27 * 16 * cinp : 27 * 256;
        hipLaunchKernelGGL(k_pack, dim3((tot + 255) / 256), dim3(256), 0, s, b.wd, cin, cout, cinp, b.wf,
                           cinp == 16 ? b.wb : nullptr);
    }
    int rc = NM_OK;
    if (mode == 0) {
        // forward, FP32 output [N][16] without activation
        if (launch_conv(cinp, EPI_F32, (const uint16_t*)x_dev, b.wf, b.bd, out_dev, nullptr, g, cout, 16, s))
            rc = NM_EHIP;
    } else if (mode == 1) {
        // backward data: out = W^T * dy as FP32 [N][16] (dy BF16 [N][16])
        if (cinp != 16) rc = NM_EINVAL;
        else if (launch_conv(16, EPI_F32, (const uint16_t*)dy_dev, b.wb, nullptr, out_dev, nullptr, g, cin, 16, s))
            rc = NM_EHIP;
    } else if (mode == 2) {
        if (launch_bwdw(cinp, (const uint16_t*)x_dev, (const uint16_t*)dy_dev, b.part, b.dw, b.db, cin, cout, g, s,
                        wave_cap))
            rc = NM_EHIP;
        else if (hipMemcpyAsync(dw_host, b.dw, nw * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                 hipMemcpyAsync(db_host, b.db, cout * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
            rc = NM_EHIP;
    } else {
        rc = NM_EINVAL;
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == NM_OK) rc = NM_EHIP;
    return rc;
}

int nm_conv3d_bf16(void* stream, int mode, const int* grid, int cinp, int cin, int cout, const void* x_dev,
                   const void* w_fp32_host, const float* bias_host, const void* dy_dev, void* out_dev,
                   float* dw_host, float* db_host)
{
    CHECK_NM(conv3d_check(grid, cinp, cin, cout));
    if (mode < 0 || mode > 2) return NM_EINVAL;
    Grid g{grid[0], grid[1], grid[2], (long)grid[0] * grid[1] * grid[2]};
    std::vector<void*> tmp;
    ConvBufs b;
    const long nw = (long)cout * cin * 27;
    int rc = NM_OK;
    if (net_alloc((void**)&b.wd, nw * 4, &tmp) || net_alloc((void**)&b.bd, 64, &tmp) ||
        net_alloc((void**)&b.wf, 27 * 16 * cinp * 2, &tmp) || net_alloc((void**)&b.wb, 27 * 256 * 2, &tmp))
        rc = NM_ENOMEM;
    if (rc == NM_OK && mode == 2) {
        const long waves = bwdw_waves(g.N / 16);
        if (net_alloc((void**)&b.part, waves * bwdw_slot_floats(cinp) * 4, &tmp) ||
            net_alloc((void**)&b.dw, nw * 4, &tmp) || net_alloc((void**)&b.db, 64, &tmp))
            rc = NM_ENOMEM;
    }
    if (rc == NM_OK)
        rc = conv3d_run((hipStream_t)stream, mode, g, cinp, cin, cout, x_dev, w_fp32_host, bias_host, dy_dev, out_dev,
                        dw_host, db_host, b, kBwdwWaves);
    for (void* q : tmp) (void)hipFree(q);
    return rc;
}

// ---------------------------------------------------------------------------
// nm_conv3d_bf16_noalloc: the same layer kernels with every device buffer of the call
// (FP32 and packed BF16 weights, bias, weight-gradient partials and sums) carved out of one
// file-scope device array, so that callers that may not allocate device memory can run
// them.  The weight-gradient pass uses at most kNoAllocWaves partial-sum slots, which keeps
// the array's size independent of the grid.  Every call on a device shares that device's
// array (kept until the process ends); calls that overlap on one device race.
// ---------------------------------------------------------------------------
constexpr long kNoAllocWaves = 256;
constexpr size_t kScratchBytes = size_t(16) << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kOffWd = 0;                                           // FP32 [16][32][27]
constexpr size_t kOffBd = kOffWd + align256(16 * 32 * 27 * 4);         // FP32 [16]
constexpr size_t kOffWf = kOffBd + align256(16 * 4);                   // BF16 [27][16][32]
constexpr size_t kOffWb = kOffWf + align256(27 * 16 * 32 * 2);         // BF16 [27][16][16]
constexpr size_t kOffDw = kOffWb + align256(27 * 256 * 2);             // FP32 [16][32][27]
constexpr size_t kOffDb = kOffDw + align256(16 * 32 * 27 * 4);         // FP32 [16]
constexpr size_t kOffPart = kOffDb + align256(16 * 4);                 // FP32 partials
constexpr size_t kScratchUsed = kOffPart + size_t(kNoAllocWaves) * bwdw_slot_floats(32) * 4;
static_assert(kScratchUsed <= kScratchBytes, "the no-allocation layout must fit the scratch array");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device, with that
// device current: the array's name is only a host-side stand-in).
int scratch_base(unsigned char** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return NM_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NM_EHIP;
        g_scratch_ptr[dev] = (unsigned char*)p;
    }
    *out = g_scratch_ptr[dev];
    return NM_OK;
}
} // namespace

int nm_conv3d_bf16_noalloc(void* stream, int mode, const int* grid, int cinp, int cin, int cout, const void* x_dev,
                           const void* w_fp32_host, const float* bias_host, const void* dy_dev, void* out_dev,
                           float* dw_host, float* db_host)
{
    CHECK_NM(conv3d_check(grid, cinp, cin, cout));
    if (mode < 0 || mode > 2) return NM_EINVAL;
    Grid g{grid[0], grid[1], grid[2], (long)grid[0] * grid[1] * grid[2]};
    unsigned char* base = nullptr;
    CHECK_NM(scratch_base(&base));
    ConvBufs b;
    b.wd = (float*)(base + kOffWd);
    b.bd = (float*)(base + kOffBd);
    b.wf = (uint16_t*)(base + kOffWf);
    b.wb = (uint16_t*)(base + kOffWb);
    b.dw = (float*)(base + kOffDw);
    b.db = (float*)(base + kOffDb);
    b.part = (float*)(base + kOffPart);
    return conv3d_run((hipStream_t)stream, mode, g, cinp, cin, cout, x_dev, w_fp32_host, bias_host, dy_dev, out_dev,
                      dw_host, db_host, b, kNoAllocWaves);
}

} // extern "C"

// ---------------------------------------------------------------------------
// Solver-side helpers (called from nm_api.hip)
// ---------------------------------------------------------------------------
namespace nm {

int warm_features(const WarmArgs& a, hipStream_t s)
{
    const long n = 3 * a.N;
    const int nb = 512;
    hipLaunchKernelGGL(k_incr_norm, dim3(nb), dim3(256), 0, s, a.ut, a.u, n, a.red);
    hipLaunchKernelGGL(k_sum_scale, dim3(1), dim3(64), 0, s, a.red, nb, n, a.scale);
    hipLaunchKernelGGL(k_features, dim3(2048), dim3(256), 0, s, a.u, a.v, a.a, a.dt, a.c2, a.phase, a.matf, a.N,
                       a.scale, a.feat);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Inference inside the solver.  The 22 material channels of the features do not change
// from step to step, so their share of layer 0 (with its bias) is computed once per
// network version and problem into l0mat (BF16 [N][16], the precision of the layer's
// output); each step then convolves only the 9 state channels (16-channel layout) and
// adds l0mat before the activation.
int warm_predict(nm_net* net, const WarmArgs& a, double* x0, hipStream_t s)
{
    Grid g{a.n1, a.n2, a.n3, a.N};
    int n3[3] = {a.n1, a.n2, a.n3};
    if (check_grid(n3) != NM_OK) return -1;
    if (!a.sfeat || !a.l0mat || !a.feat || !a.scale || !a.ut || !x0) return -1;
    if (net_workspace(net, g.N) != NM_OK) return -2;
    if (*a.l0mat_version != net->version) {
        hipLaunchKernelGGL(k_features_material, dim3(2048), dim3(256), 0, s, a.phase, a.matf, a.N, a.feat);
        const float* b0 = net->p + net->off[0] + layer_w(net, 0);
        if (launch_conv(32, EPI_BF16, a.feat, net->wf[0], b0, a.l0mat, nullptr, g, 16, 16, s)) return -2;
        *a.l0mat_version = net->version;
    }
    const long n = 3 * a.N;
    if (a.inc) {
        hipLaunchKernelGGL(k_sum_scale, dim3(1), dim3(64), 0, s, a.inc, a.inc_nb, n, a.scale);
    } else {
        hipLaunchKernelGGL(k_incr_norm, dim3(512), dim3(256), 0, s, a.ut, a.u, n, a.red);
        hipLaunchKernelGGL(k_sum_scale, dim3(1), dim3(64), 0, s, a.red, 512, n, a.scale);
    }
    // unscaled state features (left by the corrector of the previous step unless the state
    // changed since); layer 0 applies 1/s to its state share
    if (!a.sfeat_ready)
        hipLaunchKernelGGL(k_features_state, dim3(2048), dim3(256), 0, s, a.u, a.v, a.a, a.dt, a.c2, a.N, nullptr,
                           a.sfeat);
    {
        ConvExtra ex;
        ex.scale = a.scale;
        if (launch_conv(16, EPI_BF16_ACT_ADD, a.sfeat, net->wf0s, nullptr, net->act[1], a.l0mat, g, 16, 16, s, ex))
            return -2;
    }
    for (int l = 1; l < net->L; l++) {
        const float* b = net->p + net->off[l] + layer_w(net, l);
        int e;
        if (l < net->L - 1)
            e = launch_conv(16, EPI_BF16_ACT, net->act[l], net->wf[l], b, net->act[l + 1], nullptr, g, 16, 16, s);
        else
            e = launch_conv(16, EPI_F32, net->act[l], net->wf[l], b, net->pred, nullptr, g, net->cout[l], kPredStride,
                            s);
        if (e) return -2;
    }
    hipLaunchKernelGGL(k_predict, dim3(2048), dim3(256), 0, s, a.ut, net->pred, a.scale, x0, a.x0f, a.N);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int warm_target(const WarmArgs& a, const double* anext, double bdt2, float* target, hipStream_t s)
{
    hipLaunchKernelGGL(k_target, dim3(2048), dim3(256), 0, s, anext, bdt2, a.scale, target, a.N);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int warm_residual_forward(nm_net* net, const WarmArgs& a, const uint16_t* feat, double scale, const uint8_t* mask,
                          double* y, hipStream_t s)
{
    Grid g{a.n1, a.n2, a.n3, a.N};
    int n3[3] = {a.n1, a.n2, a.n3};
    if (check_grid(n3) != NM_OK) return -1;
    if (net_forward(net, g, feat, s) != NM_OK) return -2;
    hipLaunchKernelGGL(k_pred_soa, dim3(2048), dim3(256), 0, s, net->pred, scale, mask, a.N, y);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int warm_residual_backward(nm_net* net, const WarmArgs& a, const uint16_t* feat, const double* gsoa, double scale,
                           float lr, hipStream_t s)
{
    Grid g{a.n1, a.n2, a.n3, a.N};
    hipLaunchKernelGGL(k_dz_soa, dim3(2048), dim3(256), 0, s, gsoa, scale, a.N, net->dz0);
    if (net_backward(net, g, feat, s) != NM_OK) return -2;
    if (net_adam(net, lr, s) != NM_OK) return -2;
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

} // namespace nm
