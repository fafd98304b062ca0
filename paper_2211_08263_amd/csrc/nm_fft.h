// Register/LDS Stockham FFT building blocks for gfx950 (wave64).
//
// A length-L complex sequence is held by a group of G = L / R threads.  On
// entry and on exit thread t owns elements t + m * G (m = 0 .. R-1) in
// register slots v[m]; in between, radix stages exchange data through LDS.
// Each stage of radix Rs and span Ns computes, for butterfly j,
//   a_r = x[j + r L / Rs] * w^(r (j mod Ns) / (Ns Rs)),   r < Rs
//   y[(j / Ns) Ns Rs + (j mod Ns) + m Ns] = DFT_Rs(a)_m
// (the Stockham autosort formulation), so the output lands in natural order
// and the last stage writes straight back into the same register slots.
// Radix R stages come first; a final smaller radix covers L / R^k.
#pragma once
#include "nm_common.h"

namespace nm {

// In-register DFT of Rs points, natural order in and out; DIR = -1 forward, +1 inverse.
template <int Rs, int DIR, typename V> struct Dft;

template <int DIR, typename V> struct Dft<1, DIR, V> {
    static __device__ __forceinline__ void run(V*) {}
};

template <int DIR, typename V> struct Dft<2, DIR, V> {
    static __device__ __forceinline__ void run(V* a)
    {
        V t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};

template <int DIR, typename V> struct Dft<4, DIR, V> {
    static __device__ __forceinline__ void run(V* a)
    {
        V t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
        V t2 = cadd(a[1], a[3]), t3 = mul_di<DIR>(csub(a[1], a[3]));
        a[0] = cadd(t0, t2);
        a[2] = csub(t0, t2);
        a[1] = cadd(t1, t3);
        a[3] = csub(t1, t3);
    }
};

template <int DIR, typename V> struct Dft<8, DIR, V> {
    static __device__ __forceinline__ void run(V* a)
    {
        using S = decltype(a[0].x);
        const S h = (S)0.70710678118654752440084436210485;
        V e[4] = {a[0], a[2], a[4], a[6]};
        V o[4] = {a[1], a[3], a[5], a[7]};
        Dft<4, DIR, V>::run(e);
        Dft<4, DIR, V>::run(o);
        // o_m *= w8^m, w8 = exp(DIR 2 pi i / 8)
        V o1 = V{h * (o[1].x - DIR * o[1].y), h * (o[1].y + DIR * o[1].x)};
        V o2 = mul_di<DIR>(o[2]);
        V o3 = V{h * (-o[3].x - DIR * o[3].y), h * (-o[3].y + DIR * o[3].x)};
        a[0] = cadd(e[0], o[0]);
        a[4] = csub(e[0], o[0]);
        a[1] = cadd(e[1], o1);
        a[5] = csub(e[1], o1);
        a[2] = cadd(e[2], o2);
        a[6] = csub(e[2], o2);
        a[3] = cadd(e[3], o3);
        a[7] = csub(e[3], o3);
    }
};

template <int DIR, typename V> struct Dft<16, DIR, V> {
    // 16 = 4 x 4: columns, twiddles w16^(r m), rows.
    static __device__ __forceinline__ void run(V* a)
    {
        using S = decltype(a[0].x);
        V b[4][4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
#pragma unroll
            for (int q = 0; q < 4; q++) b[r][q] = a[r + 4 * q];
            Dft<4, DIR, V>::run(b[r]);
        }
        // twiddle b[r][m] by w16^(r m)
        const S c1 = (S)0.92387953251128675613, s1 = (S)0.38268343236508977173;
        const S c2 = (S)0.70710678118654752440;
#pragma unroll
        for (int r = 1; r < 4; r++)
#pragma unroll
            for (int m = 1; m < 4; m++) {
                const int e = r * m; // 1..9
                S c, s;
                switch (e) {
                case 1: c = c1; s = s1; break;
                case 2: c = c2; s = c2; break;
                case 3: c = s1; s = c1; break;
                case 4: c = 0; s = 1; break;
                case 6: c = -c2; s = c2; break;
                default: c = -c1; s = -s1; break; // e == 9: angle 9 pi / 8
                }
                V w = V{c, (S)DIR * s};
                b[r][m] = cmul(b[r][m], w);
            }
#pragma unroll
        for (int m = 0; m < 4; m++) {
            V c[4] = {b[0][m], b[1][m], b[2][m], b[3][m]};
            Dft<4, DIR, V>::run(c);
#pragma unroll
            for (int q = 0; q < 4; q++) a[m + 4 * q] = c[q];
        }
    }
};

// LDS address maps.  Lines (one group of lanes per line, stride-1 reads and
// stride-R writes in the first stages) use an XOR swizzle of the element index
// inside aligned groups of 8 (16-byte elements) or 16 (8-byte elements), so
// that both patterns spread over all banks without padding.
template <int R, int ESIZE> struct LineAddr {
    int base;
    __device__ __forceinline__ int operator()(int p) const
    {
        constexpr int S = ESIZE >= 16 ? 3 : 4, MASK = (1 << S) - 1;
        return base + (p ^ ((p >> S) & MASK));
    }
};
template <int R, int TX> struct ColAddr {
    int c;
    __device__ __forceinline__ int operator()(int p) const { return p * TX + c + p / R; }
};

// Synchronisation between the stages' LDS writes and reads.  A group that
// lives inside one wavefront (x lines: G = L / R <= 64 lanes) only needs the
// wave's LDS operations to stay in program order; columns spread over several
// waves need a block barrier.
template <bool WAVE> __device__ __forceinline__ void group_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <int L, int R> struct FftShape {
    static constexpr int G = L / R;
    static_assert(L % R == 0, "L must be a multiple of R");
};

// Twiddle sources.  The stage of span Ns and radix Rs multiplies input r of butterfly
// b (j = t + b G, k = j mod Ns) by w_L^(r k L / (Ns Rs)), w_L = exp(-2 pi i / L); the
// inverse transform takes the conjugate.
// TwTable reads the table w_L^i, i < L (in LDS); TwRegs holds the values a thread needs
// for all stages in registers, read once from the table, for kernels that run many
// transforms of one length.
template <typename V> struct TwTable {
    const V* p;
    template <int L, int Ns, int Rs> __device__ __forceinline__ V get(int, int r, int k) const
    {
        return p[r * k * (L / (Ns * Rs))];
    }
};

template <int L, int R> struct FftPlan {
    // twiddles per thread of the stages from span Ns on
    static constexpr int count_from(int Ns)
    {
        int c = 0;
        while (Ns < L) {
            const int Rs = (Ns * R <= L) ? R : (L / Ns);
            if (Ns > 1) c += (R / Rs) * (Rs - 1);
            Ns *= Rs;
        }
        return c;
    }
    static constexpr int count() { return count_from(1); }
    // index of the first twiddle of the stage of span Ns
    static constexpr int offset(int Ns) { return count() - count_from(Ns); }
};

template <int L, int R, typename V> struct TwRegs {
    using Plan = FftPlan<L, R>;
    using S = decltype(V{}.x);
    // clang vector element (an array of HIP's vector structs would stay in scratch memory)
    typedef S E __attribute__((ext_vector_type(2)));
    static constexpr int NT = Plan::count() > 0 ? Plan::count() : 1;
    E w[NT];
    template <int Ns> __device__ __forceinline__ void load_from(int t, const V* __restrict__ tab)
    {
        if constexpr (Ns < L) {
            constexpr int Rs = (Ns * R <= L) ? R : (L / Ns);
            constexpr int G = L / R, NB = R / Rs;
            if constexpr (Ns > 1) {
                constexpr int o = Plan::offset(Ns);
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    const int k = (t + b * G) & (Ns - 1);
#pragma unroll
                    for (int r = 1; r < Rs; r++) {
                        const V x = tab[r * k * (L / (Ns * Rs))];
                        w[o + b * (Rs - 1) + r - 1] = E{x.x, x.y};
                    }
                }
            }
            load_from<Ns * Rs>(t, tab);
        }
    }
    __device__ __forceinline__ void load(int t, const V* __restrict__ tab) { load_from<1>(t, tab); }
    template <int LL, int Ns, int Rs> __device__ __forceinline__ V get(int b, int r, int) const
    {
        static_assert(LL == L, "twiddle cache of another length");
        constexpr int o = Plan::offset(Ns);
        const E x = w[o + b * (Rs - 1) + r - 1];
        return V{x.x, x.y};
    }
};

// One Stockham stage (radix chosen from Ns) followed by the remaining stages.
template <int L, int R, int DIR, int Ns, bool WAVE, typename V, typename Addr, typename Tw>
__device__ __forceinline__ void fft_stage(V (&v)[R], int t, V* lds, const Addr& addr, const Tw& tw)
{
    if constexpr (Ns < L) {
        constexpr int Rs = (Ns * R <= L) ? R : (L / Ns);
        constexpr int G = L / R;
        constexpr int NB = R / Rs;
        constexpr bool first = (Ns == 1);
        constexpr bool last = (Ns * Rs == L);
        if constexpr (!first) {
#pragma unroll
            for (int m = 0; m < R; m++) v[m] = lds[addr(t + m * G)];
            group_sync<WAVE>();
        }
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int j = t + b * G;
            const int k = j & (Ns - 1);
            V a[Rs];
#pragma unroll
            for (int r = 0; r < Rs; r++) a[r] = v[b + r * NB];
            if constexpr (Ns > 1) {
#pragma unroll
                for (int r = 1; r < Rs; r++) {
                    const V w = tw.template get<L, Ns, Rs>(b, r, k);
                    a[r] = DIR > 0 ? cmulc(a[r], w) : cmul(a[r], w);
                }
            }
            Dft<Rs, DIR, V>::run(a);
            if constexpr (last) {
#pragma unroll
                for (int r = 0; r < Rs; r++) v[b + r * NB] = a[r];
            } else {
                const int base = (j / Ns) * Ns * Rs + k;
#pragma unroll
                for (int r = 0; r < Rs; r++) lds[addr(base + r * Ns)] = a[r];
            }
        }
        if constexpr (!last) group_sync<WAVE>();
        fft_stage<L, R, DIR, Ns * Rs, WAVE>(v, t, lds, addr, tw);
    }
}

// Length-L transform of the group's sequence (see file comment).  tw is a twiddle
// source (group_fft_tw) or points at the table w_L^i = exp(-2 pi i i / L), i < L.  Every
// thread of the block must call it (it contains block barriers); on exit the LDS
// area is free.
template <int L, int R, int DIR, bool WAVE = false, typename V, typename Addr, typename Tw>
__device__ __forceinline__ void group_fft_tw(V (&v)[R], int t, V* lds, const Addr& addr, const Tw& tw)
{
    // The last stage's LDS reads are followed by a sync, so no trailing one is needed.
    if constexpr (L > 1) fft_stage<L, R, DIR, 1, WAVE>(v, t, lds, addr, tw);
}
template <int L, int R, int DIR, bool WAVE = false, typename V, typename Addr>
__device__ __forceinline__ void group_fft(V (&v)[R], int t, V* lds, const Addr& addr, const V* tw)
{
    group_fft_tw<L, R, DIR, WAVE>(v, t, lds, addr, TwTable<V>{tw});
}

// Offset of the table of length L (L = 2, 4, ..., 1024) inside the packed
// twiddle array: tables are stored back to back in increasing length.
__host__ __device__ constexpr int tw_offset(int L) { return L - 2; }
constexpr int kTwiddleCount = 2046; // lengths 2 .. 1024

} // namespace nm
