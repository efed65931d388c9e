// Pencil DFTs for gfx950 in two register steps with one LDS exchange.
//
// A length n = R1 * R2 transform (n = 2^L, R2 = 2^floor(L/2), R1 = n / R2)
// is split the Cooley-Tukey way:
//   x index  j = R2 * i1 + i2,   output index  k = k1 + R1 * k2
//   X[k1 + R1 k2] = sum_i2 W_R2^(i2 k2) * W_n^(i2 k1) * sum_i1 x[R2 i1 + i2] W_R1^(i1 k1)
// Thread p (one of R2 per pencil) runs the length-R1 DFT over its stride-R2
// elements, multiplies by W_n^(p k1), and writes to LDS; after one barrier it
// gathers, for k1 = p + R2 s (s < R1/R2), the R2 values of that k1 and runs
// the length-R2 DFT.  The inverse that starts from this frequency layout is
// the mirror image (length-R2 DFTs first, then length-R1), so a product in
// frequency space followed by an inverse needs no extra exchange.
// Small DFTs are unrolled radix-2 decimation-in-time with compile-time
// twiddles; W_n twiddles come from a 1024-entry table evaluated in double
// precision at compile time and rounded once to float.
#pragma once

#include <stdint.h>

#include <type_traits>

#include <hip/hip_runtime.h>

namespace dmcr {

// Exact division by a runtime divisor d (1 <= d < 2^15) for numerators below
// 2^17: q = floor(x * M / 2^32) with M = floor(2^32 / d) + 1.  The product
// overshoots x/d by less than x/2^32 < 2^-15 < 1/d, so the floor is exact.
struct FastDivU {
    uint64_t M;
};

inline FastDivU make_fastdivu(int d) { return FastDivU{(uint64_t)((1ull << 32) / (uint64_t)d) + 1ull}; }

__device__ __forceinline__ int fdivu(int x, const FastDivU &f) { return (int)(((uint64_t)(uint32_t)x * f.M) >> 32); }

// Division by a run-time constant d >= 1, exact for every 32-bit x, after the
// round-up multiplier method of Granlund and Montgomery (PLDI 1994): with
// l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1 (which fits in 32
// bits), t = hi32(m x) gives x / d = (t + ((x - t) >> min(l, 1))) >> max(l - 1, 0).
struct DivU32 {
    uint32_t m, s1, s2;
};

inline DivU32 make_divu32(uint32_t d)
{
    int l = 0;
    while ((1ull << l) < d) ++l;
    const uint64_t m = (((1ull << 32) * ((1ull << l) - d)) / d) + 1ull;
    return DivU32{(uint32_t)m, l < 1 ? 0u : 1u, l < 1 ? 0u : (uint32_t)(l - 1)};
}

__device__ __forceinline__ uint32_t divu32(uint32_t x, const DivU32 &f)
{
    const uint32_t t = __umulhi(f.m, x);
    return (t + ((x - t) >> f.s1)) >> f.s2;
}

// ---------------------------------------------------------------------------
// compile-time trigonometry (Taylor series on [-pi, pi], double precision)
// ---------------------------------------------------------------------------
struct cf {
    float x, y;
};

constexpr double kPiD = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x)
{
    double term = x, sum = x;
    for (int k = 1; k < 40; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}

constexpr double taylor_cos(double x)
{
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 40; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}

// exp(-2 pi i m / n), exact integer reduction of m to [-n/2, n/2]
constexpr cf unit_root(int m, int n)
{
    m %= n;
    if (m < 0) m += n;
    if (2 * m > n) m -= n;
    const double a = 2.0 * kPiD * (double)m / (double)n;
    return cf{(float)taylor_cos(a), (float)(-taylor_sin(a))};
}

constexpr int kTwN = 1024;
struct TwTable {
    cf v[kTwN];
};

constexpr TwTable make_tw()
{
    TwTable t{};
    for (int m = 0; m < kTwN; ++m) t.v[m] = unit_root(m, kTwN);
    return t;
}

__constant__ const TwTable kTw = make_tw();

constexpr int clog2(int n) { return n <= 1 ? 0 : 1 + clog2(n / 2); }

constexpr int bitrev(int i, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; ++b) r = (r << 1) | ((i >> b) & 1);
    return r;
}

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 c_cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// W_n^(m) (forward) or its conjugate (inverse), m any non-negative integer, n | 1024
template <bool INV>
__device__ __forceinline__ float2 tw_n(int m, int n_log2)
{
    const cf w = kTw.v[(m << (10 - n_log2)) & (kTwN - 1)];
    return make_float2(w.x, INV ? -w.y : w.y);
}

// In-register DFT of length R (natural order in and out); INV uses exp(+2 pi i).
template <int R, bool INV>
__device__ __forceinline__ void dft_reg(float2 (&x)[R])
{
    if constexpr (R == 1) {
        return;
    } else {
        constexpr int B = clog2(R);
        float2 y[R];
        static_for<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            y[bitrev(i, B)] = x[i];
        });
        static_for<1, B + 1>([&](auto lc) {
            constexpr int len = 1 << decltype(lc)::value;
            static_for<0, R / len>([&](auto bc) {
                constexpr int i = decltype(bc)::value * len;
                static_for<0, len / 2>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    float2 v = y[i + j + len / 2];
                    if constexpr (j != 0) {
                        if constexpr (4 * j == len) {
                            v = INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
                        } else {
                            constexpr cf w = unit_root(j, len);
                            v = c_mul(v, make_float2(w.x, INV ? -w.y : w.y));
                        }
                    }
                    const float2 u = y[i + j];
                    y[i + j] = c_add(u, v);
                    y[i + j + len / 2] = c_sub(u, v);
                });
            });
        });
        static_for<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            x[i] = y[i];
        });
    }
}

// Sum of x over aligned groups of `lanes` adjacent lanes of a wave (a power of
// two, at most 64) by a fixed xor butterfly.  Partners add the same two values,
// so every lane of a group ends with the same bits, whatever the launch.
__device__ __forceinline__ double group_sum(double x, int lanes)
{
    for (int o = 1; o < lanes; o <<= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// ---------------------------------------------------------------------------
// the split of one pencil length
// ---------------------------------------------------------------------------
template <int L>
struct Split {
    static constexpr int n = 1 << L;
    static constexpr int R2 = 1 << (L / 2);
    static constexpr int R1 = n / R2;
    static constexpr int S = R1 / R2;   // 1 or 2
};

// LDS exchange slot of (k1, i2) for pencil t of a tile of T pencils; the
// (R2 + 1) row pitch keeps the gather of stage two at two passes per wave.
// Two lane orders: LANE_T (lanes walk adjacent pencils: strided axes) and
// LANE_P (lanes walk along one pencil: contiguous rows).
enum LaneOrder { LANE_T = 0, LANE_P = 1 };

template <int L, int LO>
__device__ __forceinline__ int ex_idx(int k1, int i2, int t, int T)
{
    if constexpr (LO == LANE_T)
        return (k1 * (Split<L>::R2 + 1) + i2) * T + t;
    else
        return k1 * (T * (Split<L>::R2 + 1) + 1) + t * (Split<L>::R2 + 1) + i2;
}

template <int L>
constexpr int ex_size(int T)
{
    return Split<L>::R1 * (Split<L>::R2 + 1) * T + Split<L>::R1;
}

// Two-phase exchange (S = 2 only): the R1 = 2 R2 rows of stage one cross the
// exchange R2 at a time, so a pencil needs half the LDS.  Used where the full
// exchange would cut a 256-thread tile short (n = 512).
template <int L>
constexpr bool half_ex()
{
    return Split<L>::S == 2 && ex_size<L>(256 / Split<L>::R2) > 8192;
}
template <int L>
constexpr int exh_size(int T)
{
    return half_ex<L>() ? Split<L>::R2 * (Split<L>::R2 + 1) * T + Split<L>::R2 : ex_size<L>(T);
}

// w[j] = W_n^(b j), j = 1..M-1 (w[0] = 1), n = 2^L: one table lookup for W_n^b,
// the other powers as products of two lower powers (at most 4 multiplications deep)
template <bool INV, int M>
__device__ __forceinline__ void tw_powers(int b, int L, float2 (&w)[M])
{
    w[0] = make_float2(1.f, 0.f);
    if constexpr (M > 1) w[1] = tw_n<INV>(b, L);
    static_for<2, M>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        w[j] = c_mul(w[j / 2], w[j - j / 2]);
    });
}

// Forward-structure transform.  In: v[i1] = x[R2 i1 + p].  Out: u[s][k2] =
// X[(p + R2 s) + R1 k2].  Contains two barriers (the caller must not touch
// `ex` between its calls from other threads).
// HALF: the two-phase exchange (half_ex), four barriers instead of two.
template <int L, bool INV, int LO = LANE_T, bool HALF = false>
__device__ __forceinline__ void pencil_fwd(float2 (&v)[Split<L>::R1], float2 (&u)[Split<L>::S][Split<L>::R2],
                                           float2 *ex, int p, int t, int T)
{
    using SP = Split<L>;
    float2 tw[SP::R1];
    tw_powers<INV>(p, L, tw);
    dft_reg<SP::R1, INV>(v);
    if constexpr (HALF) {
        static_assert(SP::S == 2, "the two-phase exchange splits S = 2 row sets");
        // phase s: rows k1 = s R2 + kl (kl < R2) at exchange row kl; thread p then
        // reads row p, i.e. k1 = p + R2 s, as the one-phase exchange does
        static_for<0, SP::S>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            if constexpr (s > 0) __syncthreads();
            static_for<0, SP::R2>([&](auto kc) {
                constexpr int kl = decltype(kc)::value, k1 = s * SP::R2 + kl;
                float2 w = v[k1];
                if constexpr (k1 != 0) w = c_mul(w, tw[k1]);
                ex[ex_idx<L, LO>(kl, p, t, T)] = w;
            });
            __syncthreads();
            static_for<0, SP::R2>([&](auto ic) {
                constexpr int i2 = decltype(ic)::value;
                u[s][i2] = ex[ex_idx<L, LO>(p, i2, t, T)];
            });
            dft_reg<SP::R2, INV>(u[s]);
        });
        __syncthreads();
        return;
    }
    static_for<0, SP::R1>([&](auto kc) {
        constexpr int k1 = decltype(kc)::value;
        float2 w = v[k1];
        if constexpr (k1 != 0) w = c_mul(w, tw[k1]);
        ex[ex_idx<L, LO>(k1, p, t, T)] = w;
    });
    __syncthreads();
    static_for<0, SP::S>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        const int k1 = p + SP::R2 * s;
        static_for<0, SP::R2>([&](auto ic) {
            constexpr int i2 = decltype(ic)::value;
            u[s][i2] = ex[ex_idx<L, LO>(k1, i2, t, T)];
        });
        dft_reg<SP::R2, INV>(u[s]);
    });
    __syncthreads();
}

// Mirror (inverse-structure) transform.  In: u[s][k2] = F[(p + R2 s) + R1 k2].
// Out: v[j1] = f[p + R2 j1].  Two barriers.
template <int L, bool INV, int LO = LANE_T, bool HALF = false>
__device__ __forceinline__ void pencil_mirror(float2 (&u)[Split<L>::S][Split<L>::R2], float2 (&v)[Split<L>::R1],
                                              float2 *ex, int p, int t, int T)
{
    using SP = Split<L>;
    if constexpr (HALF) {
        static_assert(SP::S == 2, "the two-phase exchange splits S = 2 row sets");
        // phase s: thread p's row k1 = p + R2 s at exchange row p; every thread
        // then reads rows kl into v[s R2 + kl], as the one-phase exchange does
        static_for<0, SP::S>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            const int k1 = p + SP::R2 * s;
            float2 tw[SP::R2];
            tw_powers<INV>(k1, L, tw);
            dft_reg<SP::R2, INV>(u[s]);
            if constexpr (s > 0) __syncthreads();
            static_for<0, SP::R2>([&](auto jc) {
                constexpr int j2 = decltype(jc)::value;
                float2 w = u[s][j2];
                if constexpr (j2 != 0) w = c_mul(w, tw[j2]);
                ex[ex_idx<L, LO>(p, j2, t, T)] = w;
            });
            __syncthreads();
            static_for<0, SP::R2>([&](auto kc) {
                constexpr int kl = decltype(kc)::value;
                v[s * SP::R2 + kl] = ex[ex_idx<L, LO>(kl, p, t, T)];
            });
        });
        dft_reg<SP::R1, INV>(v);
        __syncthreads();
        return;
    }
    static_for<0, SP::S>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        const int k1 = p + SP::R2 * s;
        float2 tw[SP::R2];
        tw_powers<INV>(k1, L, tw);
        dft_reg<SP::R2, INV>(u[s]);
        static_for<0, SP::R2>([&](auto jc) {
            constexpr int j2 = decltype(jc)::value;
            float2 w = u[s][j2];
            if constexpr (j2 != 0) w = c_mul(w, tw[j2]);
            ex[ex_idx<L, LO>(k1, j2, t, T)] = w;
        });
    });
    __syncthreads();
    static_for<0, SP::R1>([&](auto kc) {
        constexpr int k1 = decltype(kc)::value;
        v[k1] = ex[ex_idx<L, LO>(k1, p, t, T)];
    });
    dft_reg<SP::R1, INV>(v);
    __syncthreads();
}

}  // namespace dmcr
