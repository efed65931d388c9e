// FFT path of the descriptor: S_ij = (1/N^2) IDFT(conj(DFT phi_i) DFT phi_j) on the
// displacement box, and its adjoint grad_c = (1/N^2) IDFT(sum_j conj(DFT K_cj) DFT phi_j)
// where K_cj are the cotangents laid out on the box (k_build_kernels in level_ops.hip).
//
// This replaces the paper's dense mask convolution (Sec. 3.2.3, eq. convdef;
// Appendix B) by the convolution theorem, the Fourier route to correlations the
// paper points to (Sec. 3.2 and Sec. 4.1).  The transform along the contiguous
// axis is real-to-half-complex; the other axes are complex.  Transforms are
// pruned: the inverse keeps only rows |r| <= P of each axis, and the transforms
// of the cotangent boxes read only those rows.
//
// Fluctuation form.  The forward drops the zero-frequency product, so the
// transforms correlate the fields minus their means (an exact identity: the
// mean of a field lives in that one bin), and the gather adds mu_i mu_j back in
// float64 before the single rounding to float32.  The means are float64 sums
// of the float32 field taken while the first pass loads it.  Without this the
// float32 rounding of the large zero-frequency term shifts every S(r) by the
// same few 1e-8, an error that the loss gradient sums coherently over r once
// S - S* is small (Sec. 3.1 loss near its minimum).
//
// Every kernel is one pass over HBM.  Pencils are transformed in two register
// steps with one LDS exchange (fft_reg.h):
//   k_rows       contiguous-axis transform of T rows; R2 adjacent lanes walk
//                along one row, so each access is an R2-wide run of a row
//   k_cols       strided-axis transform of T adjacent pencils; lanes of a wave
//                walk adjacent pencils, so every global access is a T-wide run
//   k_axis0_fwd  axis-0 forward DFT of every channel, pair products, pruned
//                axis-0 inverse (the "reduce" step fused into the transform)
//   k_axis0_adj  axis-0 forward DFT of fields and cotangent boxes, the adjoint
//                product sum, full axis-0 inverse (in place)
#include <algorithm>

#include "dmcr_internal.h"
#include "fft_reg.h"

namespace dmcr {

namespace {

enum PassTag {
    T_R2C_LAST = 0,    // forward, contiguous axis, real -> half spectrum
    T_FWD_MID,         // forward, axis 1 (3-D), in place
    T_INV_MID_BOX,     // inverse, axis 1 (3-D), keep the |r1| <= P rows
    T_C2R_DESC,        // inverse, contiguous axis, half -> real rows of the box, into S
    T_KB_LAST,         // forward of the cotangent boxes, contiguous axis
    T_KB_MID,          // forward of the cotangent boxes, axis 1 (3-D)
    T_INV_MID,         // inverse, axis 1 (3-D), in place
    T_C2R_FULL         // inverse, contiguous axis, half -> real field
};

// Row modes of the strided passes, fixed per pass so that their loads and
// stores compile without per-element mode tests.
constexpr int col_in_mode(int tag) { return tag == T_KB_MID ? IO_BOX : IO_FULL; }
constexpr int col_out_mode(int tag) { return tag == T_INV_MID_BOX ? IO_BOX : IO_FULL; }

// tile geometry per transform length: T pencils per block, R2 threads each,
// with the LDS exchange (and the row staging) within 64 KB
template <int L>
struct Tile {
    static constexpr int R2 = Split<L>::R2;
    static constexpr int n = Split<L>::n;
    static constexpr int pick()
    {
        int T = 256 / R2;
        while (T > 1 && ex_size<L>(T) > 8192) T /= 2;
        return T;
    }
    static constexpr int T = pick();
    static constexpr int threads = R2 * T;
};

// tile geometry of the strided passes (k_cols, the axis-0 passes).  Where half_ex
// holds (n = 512) they always take the two-phase exchange, so that the compiled
// arithmetic is one and the same whatever the tile: with HX a 256-thread tile of
// 16 pencils, else Tile's 8 pencils (128 threads), which gives a small pass twice
// as many blocks.  The tile changes addresses only, so the results are
// bitwise the same; the launch picks HX for passes with enough pencils to fill the
// chip.  Elsewhere both are Tile.
template <int L, bool HX>
struct TileS {
    static constexpr int R2 = Split<L>::R2;
    static constexpr bool half = half_ex<L>();
    static constexpr int size(int T) { return half ? exh_size<L>(T) : ex_size<L>(T); }
    static constexpr int pick()
    {
        if (!HX) return Tile<L>::T;
        int T = 256 / R2;
        while (T > 1 && size(T) > 8192) T /= 2;
        return T;
    }
    static constexpr int T = pick();
    static constexpr int threads = R2 * T;
};

// a strided pass of this many pencils or more takes the 16-pencil tile where
// half_ex holds (at least 512 tiles; measured on 2-D 512^2: 4% faster at 64
// fields, 3% slower at one field, whose pass then has half as many blocks)
constexpr int64_t kHalfExMinPencils = 8192;

// Tile order of the strided passes.  Blocks are dealt to the 8 XCDs in turn
// (block i to XCD i mod 8); tile = the (i / 8)-th of XCD (i mod 8)'s contiguous
// share of the nb tiles, so the blocks that one XCD holds at a time read adjacent
// 128-byte pencil runs of the same rows instead of every eighth one.  A bijection
// of [0, nb) for any nb.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t i, uint32_t nb)
{
    const uint32_t x = i & 7u, k = i >> 3, q = nb >> 3, r = nb & 7u;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// row index e of an array that holds `mode` rows of a length-n axis, for
// transform index j; -1 if that index is not stored
__device__ __forceinline__ int row_of(int mode, int j, int n, int P)
{
    if (mode == IO_FULL) return j;
    if (mode == IO_HALF) return j <= n / 2 ? j : -1;
    const int b = (j + P) & (n - 1);  // IO_BOX / IO_DESC: box index of j
    return b <= 2 * P ? b : -1;
}

struct RowArgs {
    const void *in;
    void *out;
    int64_t nrows;
    int in_mode, out_mode, in_len, out_len, P;
    int in_valid, out_valid;  // entries of a row that hold data (the rest is pitch padding)
    int in_real, out_real;
    float scale;
    FastDivU fd_in, fd_out;
    // IO_DESC: row m = (b * npairs + p) * rows_per_pair + row of the box of pair p
    // IO_GBOX: row m = ((b * C + c) * C + j) * rows_per_pair + row of K_cj
    int npairs, auto_mask, C;
    int64_t rows_per_pair, center, Kstride, vol;
    int64_t off[kMaxPairs];
    int pi[kMaxPairs], pj[kMaxPairs];
    // IO_GBOX with St: `in` is the descriptor S and the cotangent is formed while
    // loading, G = 2 w2 (S - St) / Z, exactly as the error kernel forms it
    const double *St;
    double w2, invZ;
    // T_C2R_FULL with coarse: each real output also takes cw times its parent in
    // the next coarser level's gradient (the prolongation of the multigrid
    // adjoint); row m = (bc n0 + z) n1 + y of the fine rows, n1 = 1 in 2-D
    const float *coarse;
    float cw;
    int64_t fn0, fn1;
    // T_R2C_LAST with msum: float64 sums of the loaded field over groups of
    // mlanes lanes (mlanes / R2 whole rows of one field), one partial per group,
    // at msum[first row / (mlanes / R2)]
    double *msum;
    int mlanes;
    // IO_DESC with mu: float64 channel means [B][C]; pair (i, j) adds mu_i mu_j
    const double *mu;
};

// Box row m of the adjoint kernel K_cj (see k_build_kernels):
//   auto (c,c):  K_cc(r) = G(r) + G(-r) on the half box, K_cc(0) = 2 G(0)
//   cross (c,j): K_cj(r) = G_cj(r);   cross (j,c): K_cj(r) = G_jc(-r)
// Pairs are distinct, so at most one of them feeds a given (c, j).
struct GboxRow {
    const float *G;   // descriptor slice of the feeding pair, or null
    const double *Gt; // the same slice of the target when G is formed from S
    int kind;         // 1 auto, 2 direct, 3 mirrored
    int bi0;          // box index of the row's first entry
};

__device__ __forceinline__ GboxRow gbox_row(const RowArgs &a, uint32_t m)
{
    const uint32_t row = m % (uint32_t)a.rows_per_pair;
    uint32_t rest = m / (uint32_t)a.rows_per_pair;
    const int j = (int)(rest % (uint32_t)a.C);
    rest /= (uint32_t)a.C;
    const int c = (int)(rest % (uint32_t)a.C);
    const int64_t b = rest / (uint32_t)a.C;
    GboxRow g{nullptr, nullptr, 0, (int)row * a.in_len};
    const float *Gb = static_cast<const float *>(a.in) + b * a.Kstride;
    for (int q = 0; q < a.npairs; ++q) {
        const bool direct = a.pi[q] == c && a.pj[q] == j, mirrored = a.pi[q] == j && a.pj[q] == c;
        if (direct || mirrored) {
            g.G = Gb + a.off[q];
            if (a.St) g.Gt = a.St + b * a.Kstride + a.off[q];
            g.kind = direct ? ((c == j) ? 1 : 2) : 3;
        }
    }
    return g;
}

// box volumes are at most 1023^2 entries per row set, so box indices fit in 32 bits
__device__ __forceinline__ float gbox_value(const RowArgs &a, const GboxRow &g, int e)
{
    const int vol = (int)a.vol, center = (int)a.center;
    const int bi = g.bi0 + e;
    const int mirror = vol - 1 - bi;
    int idx = (g.kind == 2) ? bi : mirror;
    float f = 1.f;
    if (g.kind == 1) {                       // half-box entry of |r|, doubled at r = 0
        idx = (bi >= center ? bi : mirror) - center;
        f = (bi == center) ? 2.f : 1.f;
    }
    if (g.Gt) return f * (float)(2.0 * a.w2 * ((double)g.G[idx] - g.Gt[idx]) * a.invZ);
    return f * g.G[idx];
}

template <int TAG, int L, bool INV>
__global__ __launch_bounds__(256) void k_rows(RowArgs a)
{
    using SP = Split<L>;
    constexpr int T = Tile<L>::T, n = SP::n, R1 = SP::R1, R2 = SP::R2, S = SP::S;
    __shared__ float2 ex[ex_size<L>(T)];
    // lanes walk along a row: R2 adjacent lanes read R2 adjacent elements
    const int p = threadIdx.x % R2, t = threadIdx.x / R2;
    const int64_t m = (int64_t)blockIdx.x * T + t;
    const bool valid = m < a.nrows;
    float2 v[R1];
    if constexpr (TAG == T_KB_LAST) {      // input IO_GBOX, output IO_HALF (complex)
        const GboxRow g = gbox_row(a, valid ? (uint32_t)m : 0u);
        const bool any = valid && g.kind != 0;
#pragma unroll
        for (int i1 = 0; i1 < R1; ++i1) {
            const int e = row_of(IO_BOX, R2 * i1 + p, n, a.P);
            v[i1] = make_float2((any && e >= 0) ? gbox_value(a, g, e) : 0.f, 0.f);
        }
    } else if (a.in_real) {
        const float *src = static_cast<const float *>(a.in) + m * a.in_len;
#pragma unroll
        for (int i1 = 0; i1 < R1; ++i1) {
            const int e = row_of(a.in_mode, R2 * i1 + p, n, a.P);
            v[i1] = make_float2((valid && e >= 0) ? src[e] : 0.f, 0.f);
        }
        if constexpr (TAG == T_R2C_LAST) {
            if (a.msum) {
                double sm = 0.0;
#pragma unroll
                for (int i1 = 0; i1 < R1; ++i1) sm += (double)v[i1].x;
                sm = group_sum(sm, a.mlanes);
                if (valid && (threadIdx.x & (a.mlanes - 1)) == 0) a.msum[m / (a.mlanes / R2)] = sm;
            }
        }
    } else {
        const float2 *src = static_cast<const float2 *>(a.in) + m * a.in_len;
#pragma unroll
        for (int i1 = 0; i1 < R1; ++i1) {
            const int j = R2 * i1 + p;
            float2 x = make_float2(0.f, 0.f);
            if (valid) {
                if (a.in_mode == IO_HALF && j > n / 2) {
                    x = c_conj(src[n - j]);  // Hermitian completion of the half spectrum
                } else {
                    const int e = row_of(a.in_mode, j, n, a.P);
                    if (e >= 0) x = src[e];
                }
            }
            v[i1] = x;
        }
    }
    float2 u[S][R2];
    pencil_fwd<L, INV, LANE_P>(v, u, ex, p, t, T);
    if (!valid) return;
    if constexpr (TAG == T_KB_LAST) {
        float2 *dst = static_cast<float2 *>(a.out) + m * a.out_len;
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                const int k = (p + R2 * s) + R1 * k2;
                if (k <= n / 2) dst[k] = c_scale(u[s][k2], a.scale);
            }
    } else if (a.out_mode == IO_DESC) {
        // entry e of box row `row` of pair q goes to descriptor index
        // off_q + row * box + e (full box) or that minus the half-box centre
        const uint32_t row = (uint32_t)(m % a.rows_per_pair);
        const uint32_t bp = (uint32_t)(m / a.rows_per_pair);
        const int q = (int)(bp % (uint32_t)a.npairs);
        const int64_t b = bp / (uint32_t)a.npairs;
        const bool aut = (a.auto_mask >> q) & 1;
        const int64_t bi0 = (int64_t)row * a.out_len;
        float *dst = static_cast<float *>(a.out) + b * a.Kstride + a.off[q] + bi0 - (aut ? a.center : 0);
        const double mm = a.mu ? a.mu[b * a.C + a.pi[q]] * a.mu[b * a.C + a.pj[q]] : 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                const int e = row_of(IO_BOX, (p + R2 * s) + R1 * k2, n, a.P);
                if (e >= 0 && !(aut && bi0 + e < a.center)) dst[e] = (float)((double)(u[s][k2].x * a.scale) + mm);
            }
    } else if (a.out_real) {
        float *dst = static_cast<float *>(a.out) + m * a.out_len;
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                const int e = row_of(a.out_mode, (p + R2 * s) + R1 * k2, n, a.P);
                if (e >= 0) dst[e] = u[s][k2].x * a.scale;
            }
    } else {
        float2 *dst = static_cast<float2 *>(a.out) + m * a.out_len;
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                const int e = row_of(a.out_mode, (p + R2 * s) + R1 * k2, n, a.P);
                if (e >= 0) dst[e] = c_scale(u[s][k2], a.scale);
            }
    }
}

// Real rows of length n = 2^L through half-length complex transforms.
// Forward: z[m] = x[2m] + i x[2m+1], Z = DFT_{n/2}(z), then for k <= n/2
//   X[k] = E[k] + W_n^k O[k],  E = (Z[k] + conj Z[n/2-k]) / 2,  O = (Z[k] - conj Z[n/2-k]) / 2i
// (Z indices mod n/2).  Inverse (unnormalised): for k < n/2
//   Z[k] = (X[k] + conj X[n/2-k]) + i W_n^-k (X[k] - conj X[n/2-k]),  z = IDFT_{n/2}(Z),
//   x[2m] = Re z[m], x[2m+1] = Im z[m].
// W_n^(p + R2 j) = W_n^p W_n^(R2 j): one table lookup per thread, the second
// factor a compile-time constant (INV: the conjugates).
template <bool INV, int L, int J, int R2>
__device__ __forceinline__ float2 tw_split(float2 wp)
{
    constexpr cf c = unit_root(R2 * J, 1 << L);
    return c_mul(wp, make_float2(c.x, INV ? -c.y : c.y));
}

template <int TAG, int L>
__global__ __launch_bounds__(256) void k_r2c(RowArgs a)
{
    constexpr int LH = L - 1;
    using SP = Split<LH>;
    constexpr int T = Tile<LH>::T, nh = SP::n, R1 = SP::R1, R2 = SP::R2, S = SP::S;
    __shared__ float2 ex[ex_size<LH>(T)];
    const int p = threadIdx.x % R2, t = threadIdx.x / R2;
    const int64_t m = (int64_t)blockIdx.x * T + t;
    const bool valid = m < a.nrows;
    // rows past the end re-read the last row (in bounds); only stores are masked
    const float2 *src = static_cast<const float2 *>(a.in) + (valid ? m : a.nrows - 1) * (a.in_len / 2);
    float2 v[R1];
#pragma unroll
    for (int i1 = 0; i1 < R1; ++i1) v[i1] = src[R2 * i1 + p];
    if (a.msum) {
        double sm = 0.0;
#pragma unroll
        for (int i1 = 0; i1 < R1; ++i1) {
            sm += (double)v[i1].x;
            sm += (double)v[i1].y;
        }
        sm = group_sum(sm, a.mlanes);
        if (valid && (threadIdx.x & (a.mlanes - 1)) == 0) a.msum[m / (a.mlanes / R2)] = sm;
    }
    const float2 wp = tw_n<false>(p, L);
    float2 u[S][R2];
    pencil_fwd<LH, false, LANE_P>(v, u, ex, p, t, T);
    // Z in natural order for the split (pencil_fwd ended with a barrier); the row
    // pitch of R2 mod 32 float2 puts the rows that a wave touches at once (R2
    // lanes of 8 bytes each) R2 * 8 bytes apart in the 64 four-byte banks
    constexpr int pitch = nh + R2;
    static_assert(T * pitch <= ex_size<LH>(T), "natural-order rows exceed the exchange");
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) ex[t * pitch + (p + R2 * s) + R1 * k2] = u[s][k2];
    __syncthreads();
    if (!valid) return;
    float2 *dst = static_cast<float2 *>(a.out) + m * a.out_len;
    const float2 *z = ex + t * pitch;
    static_for<0, nh / R2 + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        const int k = p + R2 * j;
        if (j < nh / R2 || p == 0) {          // k <= n/2
            const float2 zk = z[k & (nh - 1)];
            const float2 zc = c_conj(z[(nh - k) & (nh - 1)]);
            const float2 E = c_scale(c_add(zk, zc), 0.5f);
            const float2 d = c_sub(zk, zc);                   // 2i O
            const float2 O = make_float2(0.5f * d.y, -0.5f * d.x);
            dst[k] = c_scale(c_add(E, c_mul(O, tw_split<false, L, j, R2>(wp))), a.scale);
        }
    });
}

template <int TAG, int L>
__global__ __launch_bounds__(256) void k_c2r(RowArgs a)
{
    constexpr int LH = L - 1;
    using SP = Split<LH>;
    constexpr int T = Tile<LH>::T, nh = SP::n, R1 = SP::R1, R2 = SP::R2, S = SP::S;
    __shared__ float2 ex[ex_size<LH>(T)];
    const int p = threadIdx.x % R2, t = threadIdx.x / R2;
    const int64_t m = (int64_t)blockIdx.x * T + t;
    const bool valid = m < a.nrows;
    const float2 *src = static_cast<const float2 *>(a.in) + (valid ? m : a.nrows - 1) * a.in_len;
    float2 xk[R1], xc[R1];
#pragma unroll
    for (int i1 = 0; i1 < R1; ++i1) {
        xk[i1] = src[R2 * i1 + p];
        xc[i1] = src[nh - R2 * i1 - p];
    }
    const float2 wp = tw_n<true>(p, L);
    float2 v[R1];
    static_for<0, R1>([&](auto ic) {
        constexpr int i1 = decltype(ic)::value;
        const float2 xm = c_conj(xc[i1]);
        const float2 e = c_add(xk[i1], xm);
        const float2 o = c_mul(c_sub(xk[i1], xm), tw_split<true, L, i1, R2>(wp));  // W_n^-k (X[k] - conj X[n/2-k])
        v[i1] = make_float2(e.x - o.y, e.y + o.x);                               // e + i o
    });
    float2 u[S][R2];
    pencil_fwd<LH, true, LANE_P>(v, u, ex, p, t, T);
    if (!valid) return;
    if constexpr (TAG == T_C2R_DESC) {
        // box row `row` of pair q: entry e goes to descriptor index off_q + row * box + e
        // (full box) or that minus the half-box centre; box indices fit in 32 bits
        const uint32_t row = (uint32_t)m % (uint32_t)a.rows_per_pair;
        const uint32_t bp = (uint32_t)m / (uint32_t)a.rows_per_pair;
        const int q = (int)(bp % (uint32_t)a.npairs);
        const int64_t b = bp / (uint32_t)a.npairs;
        const bool aut = (a.auto_mask >> q) & 1;
        const int bi0 = (int)row * a.out_len;
        const int lo = aut ? (int)a.center - bi0 : 0;   // entries e < lo are not stored
        float *dst = static_cast<float *>(a.out) + b * a.Kstride + a.off[q] + bi0 - (aut ? a.center : 0);
        const double mu2 = a.mu ? a.mu[b * a.C + a.pi[q]] * a.mu[b * a.C + a.pj[q]] : 0.0;
        const int n = 2 * nh;
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                const int mm = (p + R2 * s) + R1 * k2;
                const int e0 = row_of(IO_BOX, 2 * mm, n, a.P);
                const int e1 = row_of(IO_BOX, 2 * mm + 1, n, a.P);
                if (e0 >= 0 && e0 >= lo) dst[e0] = (float)((double)(u[s][k2].x * a.scale) + mu2);
                if (e1 >= 0 && e1 >= lo) dst[e1] = (float)((double)(u[s][k2].y * a.scale) + mu2);
            }
    } else {
        float2 *dst = static_cast<float2 *>(a.out) + m * (a.out_len / 2);
        if (TAG == T_C2R_FULL && a.coarse) {
            // outputs 2 mm and 2 mm + 1 share the parent mm of the coarse row
            const int64_t y = m % a.fn1, r = m / a.fn1;
            const int64_t z = r % a.fn0, bc = r / a.fn0;
            const int64_t h1 = a.fn1 > 1 ? a.fn1 / 2 : 1;
            const float *cr = a.coarse + ((bc * (a.fn0 / 2) + z / 2) * h1 + y / 2) * nh;
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int mm = (p + R2 * s) + R1 * k2;
                    const float2 g = c_scale(u[s][k2], a.scale);
                    const float c = cr[mm];
                    dst[mm] = make_float2(fmaf(a.cw, c, g.x), fmaf(a.cw, c, g.y));
                }
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) dst[(p + R2 * s) + R1 * k2] = c_scale(u[s][k2], a.scale);
        }
    }
}

// Strided passes: pencil locations and row indices stay in 32 bits (the host
// checks npen, nloc < 2^32 and inner < 2^24), so that a pencil needs one 64-bit
// base; rows p + R2 j of it lie a uniform stride apart and other rows (box
// modes) take a 24-bit multiply.
struct ColArgs {
    const float2 *in;
    float2 *out;
    int64_t npen, inner;  // inner = padded half-spectrum pitch hp
    int in_mode, out_mode, in_len, out_len, P;
    int h;                // columns of a pitch that hold data
    float scale;
    uint32_t inner32;
    DivU32 dv_inner;
};

template <int TAG, int L, bool INV, bool HX>
__global__ __launch_bounds__(256) void k_cols(ColArgs a)
{
    using SP = Split<L>;
    using TS = TileS<L, HX>;
    constexpr int T = TS::T, n = SP::n, R1 = SP::R1, R2 = SP::R2, S = SP::S;
    constexpr bool H = TS::half;
    constexpr int kIn = col_in_mode(TAG), kOut = col_out_mode(TAG);
    __shared__ float2 ex[TS::size(T)];
    const int t = threadIdx.x % T, p = threadIdx.x / T;
    const int64_t m = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * T + t;
    const uint32_t mu = m < a.npen ? (uint32_t)m : 0u;
    const uint32_t o = divu32(mu, a.dv_inner);
    const uint32_t i = mu - o * a.inner32;
    const bool valid = m < a.npen && (int)i < a.h;
    const size_t inner = a.inner32;
    const float2 *src = a.in + (size_t)o * a.in_len * inner + i;
    float2 v[R1];
    if constexpr (kIn == IO_FULL) {
        const float2 *sp = src + (size_t)p * inner;
#pragma unroll
        for (int i1 = 0; i1 < R1; ++i1)
            v[i1] = valid ? sp[(size_t)(R2 * i1) * inner] : make_float2(0.f, 0.f);
    } else {
#pragma unroll
        for (int i1 = 0; i1 < R1; ++i1) {
            const int e = row_of(kIn, R2 * i1 + p, n, a.P);
            v[i1] = (valid && e >= 0) ? src[__umul24((uint32_t)e, a.inner32)] : make_float2(0.f, 0.f);
        }
    }
    float2 u[S][R2];
    pencil_fwd<L, INV, LANE_T, H>(v, u, ex, p, t, T);
    if (!valid) return;
    float2 *dst = a.out + (size_t)o * a.out_len * inner + i;
    if constexpr (kOut == IO_FULL) {
        float2 *dp = dst + (size_t)p * inner;
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) dp[(size_t)(R2 * s + R1 * k2) * inner] = c_scale(u[s][k2], a.scale);
    } else {
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                const int e = row_of(kOut, (p + R2 * s) + R1 * k2, n, a.P);
                if (e >= 0) dst[__umul24((uint32_t)e, a.inner32)] = c_scale(u[s][k2], a.scale);
            }
    }
}

struct Axis0Args {
    float2 *X;          // [B][C][n][inner] partial spectra (axes 1.. transformed)
    const float2 *KB;   // adjoint: [B][C*C][box][inner]
    float2 *Y;          // forward: [B][npairs][box][inner]
    int64_t inner, nloc;  // nloc = B * inner pencil locations
    int P, box, npairs;
    int h, hp;            // data columns of each padded half-spectrum row
    int pair_of[kMaxChannels * kMaxChannels];  // (i, j) -> pair index or -1
    float scale;
    uint32_t inner32;
    DivU32 dv_inner, dv_hp;
    // forward: the first nmean blocks form the float64 field means
    // mu[f] = (sum of msum[f][0 .. mparts)) * invN instead of a pencil tile
    const double *msum;
    double *mu;
    int64_t mparts;
    double invN;
    uint32_t nmean;
};

// pencil location m -> (field b, column i); false for padding columns and m past the end
struct Axis0Loc {
    uint32_t b, i;
    bool valid;
};

__device__ __forceinline__ Axis0Loc axis0_loc(const Axis0Args &a, int64_t m)
{
    const uint32_t mu = m < a.nloc ? (uint32_t)m : 0u;
    Axis0Loc l;
    l.b = divu32(mu, a.dv_inner);
    l.i = mu - l.b * a.inner32;
    const uint32_t col = l.i - divu32(l.i, a.dv_hp) * (uint32_t)a.hp;
    l.valid = m < a.nloc && (int)col < a.h;
    return l;
}

// rows p + R2 i1 (i1 < R1) of a full pencil that starts at `base`
template <int R1, int R2>
__device__ __forceinline__ void load_rows(float2 (&v)[R1], const float2 *base, int p, size_t inner, bool valid)
{
    const float2 *sp = base + (size_t)p * inner;
#pragma unroll
    for (int i1 = 0; i1 < R1; ++i1) v[i1] = valid ? sp[(size_t)(R2 * i1) * inner] : make_float2(0.f, 0.f);
}

// mu[f] = (sum of field f's mparts partial sums) * invN, float64, by the first NT
// threads of one block (NT a power of two that depends on the level only, not on
// the block size the launch picked): thread t adds the partials t, t + NT, ... in
// index order, eight loads in flight, then a fixed tree in red[NT].  The same bits
// for a field in any batch.  The other threads of the block only take the barriers.
template <int NT>
__device__ __forceinline__ void field_mean(const Axis0Args &a, uint32_t f, double *red)
{
    const double *pf = a.msum + (int64_t)f * a.mparts;
    if (threadIdx.x < NT) {
        double sm = 0.0;
        for (int64_t j0 = threadIdx.x; j0 < a.mparts; j0 += 8 * NT) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t j = j0 + (int64_t)u * NT;
                v[u] = j < a.mparts ? pf[j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) sm += v[u];
        }
        red[threadIdx.x] = sm;
    }
    __syncthreads();
#pragma unroll
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.mu[f] = red[0] * a.invN;
}

template <int L, int C, bool HX>
__global__ __launch_bounds__(256) void k_axis0_fwd(Axis0Args a)
{
    using SP = Split<L>;
    using TS = TileS<L, HX>;
    constexpr int T = TS::T, n = SP::n, R1 = SP::R1, R2 = SP::R2, S = SP::S;
    constexpr bool H = TS::half;
    __shared__ float2 ex[TS::size(T)];
    // the means' tree width: the one-phase tile's thread count, whichever tile runs
    constexpr int NTM = TileS<L, false>::threads;
    static_assert(sizeof(float2) == sizeof(double) && TS::size(T) >= NTM && TS::threads >= NTM,
                  "the exchange holds the means' float64 tree");
    if (blockIdx.x < a.nmean) {   // block-uniform: a means block does no pencil work
        field_mean<NTM>(a, blockIdx.x, reinterpret_cast<double *>(ex));
        return;
    }
    const int t = threadIdx.x % T, p = threadIdx.x / T;
    const Axis0Loc loc = axis0_loc(a, (int64_t)xcd_tile(blockIdx.x - a.nmean, gridDim.x - a.nmean) * T + t);
    const size_t inner = a.inner32;
    float2 X[C][S][R2];
    static_for<0, C>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        float2 v[R1];
        load_rows<R1, R2>(v, a.X + ((size_t)loc.b * C + c) * n * inner + loc.i, p, inner, loc.valid);
        pencil_fwd<L, false, LANE_T, H>(v, X[c], ex, p, t, T);
    });
    static_for<0, C>([&](auto ic) {
        constexpr int ci = decltype(ic)::value;
        static_for<ci, C>([&](auto jc) {
            constexpr int cj = decltype(jc)::value;
            const int q = a.pair_of[ci * kMaxChannels + cj];
            if (q >= 0) {
                float2 w[S][R2];
#pragma unroll
                for (int s = 0; s < S; ++s)
#pragma unroll
                    for (int k = 0; k < R2; ++k) w[s][k] = c_scale(c_cmul(X[ci][s][k], X[cj][s][k]), a.scale);
                // the zero frequency of the field (column 0, row k0 = 0): the product of
                // the means, added back in float64 by the gather
                if (loc.i == 0 && p == 0) w[0][0] = make_float2(0.f, 0.f);
                float2 out[R1];
                pencil_mirror<L, true, LANE_T, H>(w, out, ex, p, t, T);
                if (loc.valid) {
                    float2 *dst = a.Y + ((size_t)loc.b * a.npairs + q) * a.box * inner + loc.i;
#pragma unroll
                    for (int j1 = 0; j1 < R1; ++j1) {
                        const int e = row_of(IO_BOX, p + R2 * j1, n, a.P);
                        if (e >= 0) dst[__umul24((uint32_t)e, a.inner32)] = out[j1];
                    }
                }
            }
        });
    });
}

template <int L, int C, bool HX>
__global__ __launch_bounds__(256) void k_axis0_adj(Axis0Args a)
{
    using SP = Split<L>;
    using TS = TileS<L, HX>;
    constexpr int T = TS::T, n = SP::n, R1 = SP::R1, R2 = SP::R2, S = SP::S;
    constexpr bool H = TS::half;
    __shared__ float2 ex[TS::size(T)];
    const int t = threadIdx.x % T, p = threadIdx.x / T;
    const Axis0Loc loc = axis0_loc(a, (int64_t)xcd_tile(blockIdx.x, gridDim.x) * T + t);
    const size_t inner = a.inner32;
    float2 X[C][S][R2];
    static_for<0, C>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        float2 v[R1];
        load_rows<R1, R2>(v, a.X + ((size_t)loc.b * C + c) * n * inner + loc.i, p, inner, loc.valid);
        pencil_fwd<L, false, LANE_T, H>(v, X[c], ex, p, t, T);
    });
    static_for<0, C>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        float2 acc[S][R2];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < R2; ++k) acc[s][k] = make_float2(0.f, 0.f);
        static_for<0, C>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const float2 *kb = a.KB + ((size_t)loc.b * C * C + c * C + j) * a.box * inner + loc.i;
            float2 v[R1];
#pragma unroll
            for (int i1 = 0; i1 < R1; ++i1) {
                const int e = row_of(IO_BOX, R2 * i1 + p, n, a.P);
                v[i1] = (loc.valid && e >= 0) ? kb[__umul24((uint32_t)e, a.inner32)] : make_float2(0.f, 0.f);
            }
            float2 K[S][R2];
            pencil_fwd<L, false, LANE_T, H>(v, K, ex, p, t, T);
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k = 0; k < R2; ++k) acc[s][k] = c_add(acc[s][k], c_cmul(K[s][k], X[j][s][k]));
        });
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < R2; ++k) acc[s][k] = c_scale(acc[s][k], a.scale);
        float2 out[R1];
        pencil_mirror<L, true, LANE_T, H>(acc, out, ex, p, t, T);
        if (loc.valid) {
            float2 *dp = a.X + ((size_t)loc.b * C + c) * n * inner + loc.i + (size_t)p * inner;
#pragma unroll
            for (int j1 = 0; j1 < R1; ++j1) dp[(size_t)(R2 * j1) * inner] = out[j1];
        }
    });
}

int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// lanes of the contiguous-axis forward that hold one partial sum of the mean:
// R2 lanes per row, whole rows of one field, at most a wave
int mean_lanes(const Plan &p, int l)
{
    const LevelPlan &L = p.lv[l];
    const int nl = L.n[p.ndim - 1];
    const int LL = nl >= 4 ? ilog2(nl) - 1 : ilog2(nl);   // packed real rows use the half length
    const int R2 = 1 << (LL / 2);
    const int64_t rpc = L.N / nl;                          // rows per field
    return (int)std::min<int64_t>(64, rpc * R2);
}


const char *const kPassName[] = {"r2c_last", "fwd_mid", "inv_mid_box", "c2r_last_desc",
                                 "kb_last", "kb_mid", "inv_mid", "c2r_last"};

// threads and tile per L (host mirror of Tile<L>)
struct TileInfo {
    int T, threads;
};

template <int L>
TileInfo tile_info()
{
    return TileInfo{Tile<L>::T, Tile<L>::threads};
}

// the strided passes' geometry, two-phase exchange (HX) or not
template <int L>
TileInfo tile_info_s(bool hx)
{
    return hx ? TileInfo{TileS<L, true>::T, TileS<L, true>::threads} : TileInfo{TileS<L, false>::T, TileS<L, false>::threads};
}

TileInfo tile_of_s(int L, bool hx)
{
    switch (L) {
    case 0: return tile_info_s<0>(hx);
    case 1: return tile_info_s<1>(hx);
    case 2: return tile_info_s<2>(hx);
    case 3: return tile_info_s<3>(hx);
    case 4: return tile_info_s<4>(hx);
    case 5: return tile_info_s<5>(hx);
    case 6: return tile_info_s<6>(hx);
    case 7: return tile_info_s<7>(hx);
    case 8: return tile_info_s<8>(hx);
    case 9: return tile_info_s<9>(hx);
    default: return tile_info_s<10>(hx);
    }
}

bool half_ex_of(int L)
{
    switch (L) {
    case 1: return half_ex<1>();
    case 2: return half_ex<2>();
    case 3: return half_ex<3>();
    case 4: return half_ex<4>();
    case 5: return half_ex<5>();
    case 6: return half_ex<6>();
    case 7: return half_ex<7>();
    case 8: return half_ex<8>();
    case 9: return half_ex<9>();
    case 10: return half_ex<10>();
    }
    return false;
}

TileInfo tile_of(int L)
{
    switch (L) {
    case 0: return tile_info<0>();
    case 1: return tile_info<1>();
    case 2: return tile_info<2>();
    case 3: return tile_info<3>();
    case 4: return tile_info<4>();
    case 5: return tile_info<5>();
    case 6: return tile_info<6>();
    case 7: return tile_info<7>();
    case 8: return tile_info<8>();
    case 9: return tile_info<9>();
    default: return tile_info<10>();
    }
}

#define DMCR_L_CASES(MACRO) \
    MACRO(1) MACRO(2) MACRO(3) MACRO(4) MACRO(5) MACRO(6) MACRO(7) MACRO(8) MACRO(9) MACRO(10)

template <int TAG, bool INV>
hipError_t rows_launch(int L, const RowArgs &a, double bytes, hipStream_t st)
{
    if (TAG == T_KB_LAST && (a.in_mode != IO_GBOX || a.out_mode != IO_HALF || a.out_real || a.vol >= (int64_t(1) << 31)))
        return hipErrorInvalidValue;
    const TileInfo ti = tile_of(L);
    const dim3 g((unsigned)((a.nrows + ti.T - 1) / ti.T)), b(ti.threads);
    switch (L) {
#define C_(LL) \
    case LL: return launch(kPassName[TAG], bytes, k_rows<TAG, LL, INV>, g, b, 0, st, a);
        DMCR_L_CASES(C_)
#undef C_
    }
    return hipErrorInvalidValue;
}

// packed real transforms (L >= 2): tile geometry of the half length
template <int TAG, bool C2R>
hipError_t real_launch(int L, const RowArgs &a, double bytes, hipStream_t st)
{
    if (C2R && (a.out_mode == IO_DESC) != (TAG == T_C2R_DESC)) return hipErrorInvalidValue;
    if (TAG == T_C2R_DESC && (a.nrows >= (int64_t(1) << 32) || a.center >= (int64_t(1) << 31)))
        return hipErrorInvalidValue;
    const TileInfo ti = tile_of(L - 1);
    const dim3 g((unsigned)((a.nrows + ti.T - 1) / ti.T)), b(ti.threads);
    switch (L) {
#define C_(LL)                                                                              \
    case LL:                                                                                \
        if constexpr (LL >= 2)                                                              \
            return C2R ? launch(kPassName[TAG], bytes, k_c2r<TAG, LL>, g, b, 0, st, a)     \
                       : launch(kPassName[TAG], bytes, k_r2c<TAG, LL>, g, b, 0, st, a);    \
        break;
        DMCR_L_CASES(C_)
#undef C_
    }
    return hipErrorInvalidValue;
}

template <int TAG, bool INV>
hipError_t cols_launch(int L, const ColArgs &a, double bytes, hipStream_t st)
{
    if (a.in_mode != col_in_mode(TAG) || a.out_mode != col_out_mode(TAG)) return hipErrorInvalidValue;
    if (a.npen >= (int64_t(1) << 32) || a.inner >= (int64_t(1) << 24)) return hipErrorInvalidValue;
    const bool hx = half_ex_of(L) && a.npen >= kHalfExMinPencils;
    const TileInfo ti = tile_of_s(L, hx);
    const dim3 g((unsigned)((a.npen + ti.T - 1) / ti.T)), b(ti.threads);
    switch (L) {
#define C_(LL)                                                                                      \
    case LL:                                                                                        \
        if constexpr (half_ex<LL>())                                                                \
            if (hx) return launch(kPassName[TAG], bytes, k_cols<TAG, LL, INV, true>, g, b, 0, st, a); \
        return launch(kPassName[TAG], bytes, k_cols<TAG, LL, INV, false>, g, b, 0, st, a);
        DMCR_L_CASES(C_)
#undef C_
    }
    return hipErrorInvalidValue;
}

template <int C>
hipError_t axis0_launch_c(bool adj, int L, const Axis0Args &a, double bytes, hipStream_t st)
{
    const bool hx = half_ex_of(L) && a.nloc >= kHalfExMinPencils;
    const TileInfo ti = tile_of_s(L, hx);
    const dim3 g((unsigned)((a.nloc + ti.T - 1) / ti.T + (adj ? 0 : a.nmean))), b(ti.threads);
    switch (L) {
#define C_(LL)                                                                                   \
    case LL:                                                                                     \
        if constexpr (half_ex<LL>())                                                             \
            if (hx)                                                                              \
                return adj ? launch("axis0_adj", bytes, k_axis0_adj<LL, C, true>, g, b, 0, st, a) \
                           : launch("axis0_fwd", bytes, k_axis0_fwd<LL, C, true>, g, b, 0, st, a); \
        return adj ? launch("axis0_adj", bytes, k_axis0_adj<LL, C, false>, g, b, 0, st, a)       \
                   : launch("axis0_fwd", bytes, k_axis0_fwd<LL, C, false>, g, b, 0, st, a);
        DMCR_L_CASES(C_)
#undef C_
    }
    return hipErrorInvalidValue;
}

hipError_t axis0_launch(int C, bool adj, int L, Axis0Args a, double bytes, hipStream_t st)
{
    if (a.nloc >= (int64_t(1) << 32) || a.inner >= (int64_t(1) << 24)) return hipErrorInvalidValue;
    a.inner32 = (uint32_t)a.inner;
    a.dv_inner = make_divu32((uint32_t)a.inner);
    a.dv_hp = make_divu32((uint32_t)a.hp);
    switch (C) {
    case 1: return axis0_launch_c<1>(adj, L, a, bytes, st);
    case 2: return axis0_launch_c<2>(adj, L, a, bytes, st);
    case 3: return axis0_launch_c<3>(adj, L, a, bytes, st);
    default: return axis0_launch_c<4>(adj, L, a, bytes, st);
    }
}

RowArgs row_args(const void *in, void *out, int64_t nrows, int in_mode, int in_len, int out_mode, int out_len,
                 int P, bool in_real, bool out_real, float scale)
{
    RowArgs a{};
    a.in = in;
    a.out = out;
    a.nrows = nrows;
    a.in_mode = in_mode;
    a.in_len = in_len;
    a.out_mode = out_mode;
    a.out_len = out_len;
    a.P = P;
    a.in_real = in_real;
    a.out_real = out_real;
    a.scale = scale;
    a.in_valid = in_len;
    a.out_valid = out_len;
    a.fd_in = make_fastdivu(in_len);
    a.fd_out = make_fastdivu(out_len);
    return a;
}

double row_bytes(const RowArgs &a)
{
    return (double)a.nrows * a.in_valid * (a.in_real ? 4 : 8) + (double)a.nrows * a.out_valid * (a.out_real ? 4 : 8);
}

ColArgs col_args(const float2 *in, float2 *out, int64_t npen, int64_t inner, int in_mode, int in_len, int out_mode,
                 int out_len, int P)
{
    ColArgs a{};
    a.in = in;
    a.out = out;
    a.npen = npen;
    a.inner = inner;
    a.in_mode = in_mode;
    a.in_len = in_len;
    a.out_mode = out_mode;
    a.out_len = out_len;
    a.P = P;
    a.h = (int)inner;
    a.scale = 1.f;
    a.inner32 = (uint32_t)inner;
    a.dv_inner = make_divu32((uint32_t)inner);
    return a;
}

double col_bytes(const ColArgs &a) { return (double)a.npen / a.inner * a.h * (a.in_len + a.out_len) * 8; }

#define TRY_HIP(expr)                         \
    do {                                      \
        hipError_t _e = (expr);               \
        if (_e != hipSuccess) return _e;      \
    } while (0)

}  // namespace

bool fft_supported(const Plan &p, int l)
{
    const LevelPlan &L = p.lv[l];
    for (int a = 0; a < p.ndim; ++a)
        if (L.n[a] > kMaxFft || L.n[a] < 2) return false;
    return p.C <= 4;
}

int64_t fft_mean_parts(const Plan &p, int l)
{
    const LevelPlan &L = p.lv[l];
    if (plane_supported(p, l)) return (int64_t)L.n[0] * plane_waves(p, l);
    const int nl = L.n[p.ndim - 1];
    const int LL = nl >= 4 ? ilog2(nl) - 1 : ilog2(nl);
    const int R2 = 1 << (LL / 2);
    return L.N / nl / (mean_lanes(p, l) / R2);
}

// Half spectrum of every channel, transformed along every axis except 0:
// X = DFT_{1..d-1}(phi) (the contiguous axis real-to-half-complex).
hipError_t fft_spectrum_level(const Plan &p, int l, const float *phi, const Ws &ws, hipStream_t st, bool fused,
                              double *msum)
{
    const LevelPlan &L = p.lv[l];
    const int B = p.B, C = p.C;
    float2 *X = ws.at<float2>(L.X);
    if (fused && plane_supported(p, l)) return plane_forward(p, l, phi, X, st, msum);   // both axes in one pass
    const int nl = L.n[p.ndim - 1];
    const int64_t rows = (p.ndim == 2) ? (int64_t)B * C * L.n[0] : (int64_t)B * C * L.n[0] * L.n[1];
    RowArgs r = row_args(phi, X, rows, IO_FULL, nl, IO_HALF, L.hp, 0, true, false, 1.f);
    r.out_valid = L.h;
    if (msum) {
        r.msum = msum;
        r.mlanes = mean_lanes(p, l);
    }
    if (nl >= 4)
        TRY_HIP((real_launch<T_R2C_LAST, false>(ilog2(nl), r, row_bytes(r), st)));
    else
        TRY_HIP((rows_launch<T_R2C_LAST, false>(ilog2(nl), r, row_bytes(r), st)));
    if (p.ndim == 3) {
        ColArgs c = col_args(X, X, (int64_t)B * C * L.n[0] * L.hp, L.hp, IO_FULL, L.n[1], IO_FULL, L.n[1], 0);
        c.h = L.h;
        TRY_HIP((cols_launch<T_FWD_MID, false>(ilog2(L.n[1]), c, col_bytes(c), st)));
    }
    return hipSuccess;
}

hipError_t fft_forward_level(const Plan &p, int l, const float *phi, float *S, const Ws &ws, hipStream_t st,
                             hipEvent_t x_free)
{
    const LevelPlan &L = p.lv[l];
    const int B = p.B, C = p.C;
    double *msum = ws.at<double>(L.msum);
    double *mu = ws.at<double>(L.mu);
    TRY_HIP(fft_spectrum_level(p, l, phi, ws, st, true, msum));
    float2 *X = ws.at<float2>(L.X);
    float2 *Y = ws.at<float2>(L.Y);
    const int n0 = L.n[0];
    const int64_t inner = (p.ndim == 2) ? L.hp : (int64_t)L.n[1] * L.hp;
    const int64_t inner_valid = inner / L.hp * L.h;
    const double invN = 1.0 / (double)L.N;

    Axis0Args a{};
    a.h = L.h;
    a.hp = L.hp;
    a.X = X;
    a.Y = Y;
    a.inner = inner;
    a.nloc = (int64_t)B * inner;
    a.P = L.P;
    a.box = L.box;
    a.npairs = p.npairs;
    for (int k = 0; k < kMaxChannels * kMaxChannels; ++k) a.pair_of[k] = -1;
    for (int q = 0; q < p.npairs; ++q) a.pair_of[p.pi[q] * kMaxChannels + p.pj[q]] = q;
    a.scale = (float)(invN * invN);
    a.msum = msum;
    a.mu = mu;
    a.mparts = L.mparts;
    a.invN = invN;
    a.nmean = (uint32_t)(B * C);
    const double bytes0 = (double)B * C * n0 * inner_valid * 8 + (double)B * p.npairs * L.box * inner_valid * 8 +
                          (double)B * C * L.mparts * 8;
    TRY_HIP(axis0_launch(C, false, ilog2(n0), a, bytes0, st));
    if (x_free) TRY_HIP(hipEventRecord(x_free, st));

    // remaining inverse axes, pruned, then scatter into descriptor order
    const float2 *last_in = Y;
    int64_t rows_per_pair = L.box;
    if (p.ndim == 3) {
        float2 *Y2 = ws.at<float2>(L.Y2);
        ColArgs c = col_args(Y, Y2, (int64_t)B * p.npairs * L.box * L.hp, L.hp, IO_FULL, L.n[1], IO_BOX, L.box, L.P);
        c.h = L.h;
        TRY_HIP((cols_launch<T_INV_MID_BOX, true>(ilog2(L.n[1]), c, col_bytes(c), st)));
        last_in = Y2;
        rows_per_pair = (int64_t)L.box * L.box;
    }
    const int nl = L.n[p.ndim - 1];
    RowArgs d = row_args(last_in, S, (int64_t)B * p.npairs * rows_per_pair, IO_HALF, L.hp, IO_DESC, L.box, L.P,
                         false, true, 1.f);
    d.in_valid = L.h;
    d.npairs = p.npairs;
    d.rows_per_pair = rows_per_pair;
    d.Kstride = p.K;
    int64_t boxvol = 1;
    for (int a2 = 0; a2 < p.ndim; ++a2) boxvol *= L.box;
    d.center = (boxvol - 1) / 2;
    d.auto_mask = 0;
    d.mu = mu;
    d.C = C;
    for (int q = 0; q < p.npairs; ++q) {
        d.off[q] = L.off[q];
        d.pi[q] = p.pi[q];
        d.pj[q] = p.pj[q];
        if (p.pi[q] == p.pj[q]) d.auto_mask |= 1 << q;
    }
    const double dbytes = (double)d.nrows * L.h * 8 + (double)d.nrows * L.box * 4;
    if (nl >= 4) return real_launch<T_C2R_DESC, true>(ilog2(nl), d, dbytes, st);
    return rows_launch<T_C2R_DESC, true>(ilog2(nl), d, dbytes, st);
}

bool fft_fused_prolong(const Plan &p, int l)
{
    return p.lv[l].path == DMCR_PATH_FFT && (plane_supported(p, l) || p.lv[l].n[p.ndim - 1] >= 4);
}

hipError_t fft_adjoint_level(const Plan &p, int l, const float *phi, const float *G, float *grad,
                             bool have_spectrum, const Ws &ws, hipStream_t st, hipStream_t st_spec, hipEvent_t x_free,
                             hipEvent_t spec_done, const double *St, const float *coarse, hipEvent_t coarse_ready)
{
    if (coarse && !fft_fused_prolong(p, l)) return hipErrorInvalidValue;
    const LevelPlan &L = p.lv[l];
    const int B = p.B, C = p.C, CC = C * C;
    float2 *KB1 = ws.at<float2>(L.KB1);
    const int nl = L.n[p.ndim - 1];
    const float2 *KBaxis0;
    // adjoint kernels K_cj built from G while loading, transformed along the contiguous axis
    const int64_t rows_per_box = (p.ndim == 2) ? L.box : (int64_t)L.box * L.box;
    RowArgs r = row_args(G, KB1, (int64_t)B * CC * rows_per_box, IO_GBOX, L.box, IO_HALF, L.hp, L.P, true, false, 1.f);
    r.out_valid = L.h;
    r.rows_per_pair = rows_per_box;
    r.C = C;
    r.npairs = p.npairs;
    r.Kstride = p.K;
    r.vol = rows_per_box * L.box;
    r.center = (r.vol - 1) / 2;
    for (int q = 0; q < p.npairs; ++q) {
        r.off[q] = L.off[q];
        r.pi[q] = p.pi[q];
        r.pj[q] = p.pj[q];
    }
    if (St) {
        r.St = St;
        r.w2 = p.w[l] * p.w[l];
        r.invZ = 1.0 / p.Z;
    }
    const double kb_bytes =
        (double)B * (p.lvl_off[l + 1] - p.lvl_off[l]) * (St ? 12 : 4) + (double)r.nrows * L.h * 8;
    TRY_HIP((rows_launch<T_KB_LAST, false>(ilog2(nl), r, kb_bytes, st)));
    if (p.ndim == 2) {
        KBaxis0 = KB1;
    } else {
        float2 *KB2 = ws.at<float2>(L.KB2);
        ColArgs c = col_args(KB1, KB2, (int64_t)B * CC * L.box * L.hp, L.hp, IO_BOX, L.box, IO_FULL, L.n[1], L.P);
        c.h = L.h;
        TRY_HIP((cols_launch<T_KB_MID, false>(ilog2(L.n[1]), c, col_bytes(c), st)));
        KBaxis0 = KB2;
    }
    if (!have_spectrum) {
        if (st_spec) {
            if (x_free) TRY_HIP(hipStreamWaitEvent(st_spec, x_free, 0));
            // a plane workgroup takes a whole CU's LDS, so the fused pass would
            // not share the CUs with the cotangent transforms it overlaps
            TRY_HIP(fft_spectrum_level(p, l, phi, ws, st_spec, false));
            TRY_HIP(hipEventRecord(spec_done, st_spec));
            TRY_HIP(hipStreamWaitEvent(st, spec_done, 0));
        } else {
            TRY_HIP(fft_spectrum_level(p, l, phi, ws, st));
        }
    }
    float2 *X = ws.at<float2>(L.X);
    const int n0 = L.n[0];
    const int64_t inner = (p.ndim == 2) ? L.hp : (int64_t)L.n[1] * L.hp;
    const int64_t inner_valid = inner / L.hp * L.h;
    const double invN = 1.0 / (double)L.N;
    Axis0Args a{};
    a.h = L.h;
    a.hp = L.hp;
    a.X = X;
    a.KB = KBaxis0;
    a.inner = inner;
    a.nloc = (int64_t)B * inner;
    a.P = L.P;
    a.box = L.box;
    a.scale = (float)(invN * invN);
    const double bytes0 = 2.0 * B * C * n0 * inner_valid * 8 + (double)B * CC * L.box * inner_valid * 8;
    TRY_HIP(axis0_launch(C, true, ilog2(n0), a, bytes0, st));
    if (coarse && coarse_ready) TRY_HIP(hipStreamWaitEvent(st, coarse_ready, 0));
    if (plane_supported(p, l)) return plane_inverse(p, l, X, grad, st, coarse);   // both axes in one pass
    if (p.ndim == 3) {
        ColArgs c = col_args(X, X, (int64_t)B * C * n0 * L.hp, L.hp, IO_FULL, L.n[1], IO_FULL, L.n[1], 0);
        c.h = L.h;
        TRY_HIP((cols_launch<T_INV_MID, true>(ilog2(L.n[1]), c, col_bytes(c), st)));
    }
    const int64_t rows = (p.ndim == 2) ? (int64_t)B * C * n0 : (int64_t)B * C * n0 * L.n[1];
    RowArgs o = row_args(X, grad, rows, IO_HALF, L.hp, IO_FULL, nl, 0, false, true, 1.f);
    o.in_valid = L.h;
    double obytes = row_bytes(o);
    if (coarse) {
        o.coarse = coarse;
        o.cw = p.ndim == 2 ? 0.25f : 0.125f;
        o.fn0 = n0;
        o.fn1 = (p.ndim == 2) ? 1 : L.n[1];
        obytes += (double)rows * nl * 4 / (1 << p.ndim);   // the coarse level: 2^-d of the voxels
    }
    if (nl >= 4) return real_launch<T_C2R_FULL, true>(ilog2(nl), o, obytes, st);
    return rows_launch<T_C2R_FULL, true>(ilog2(nl), o, obytes, st);
}

}  // namespace dmcr
