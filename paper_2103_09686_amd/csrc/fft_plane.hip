// Fused two-axis transforms of square planes on 3-D levels: the contiguous axis
// (real <-> half complex) and axis 1 in one pass over HBM, so that a 3-D
// transform costs two passes (this one and the axis-0 pass) instead of three.
//
// One workgroup owns one plane of n x n reals (n = 2^L, 32 <= n <= 256) and
// its half spectrum of n rows by n/2 + 1 complex columns.  At n = 256 that half
// spectrum (264 KB) is larger than the 160 KB of LDS, so the axis-1 transform is
// split once: the forward by decimation in frequency,
//   X[2m] = DFT_{n/2}(a + b)[m],   X[2m + 1] = DFT_{n/2}((a - b) W_n^r)[m],
// a and b being rows r and r + n/2, and the inverse by the mirror decimation in
// time.  Each half-length column set is staged through LDS in turn while the
// other waits in registers.  Columns 0 and n/2 of the contiguous-axis transform
// are real along axis 1; they travel as one complex column Z = X_0 + i X_{n/2}
// and are separated after the column transform with the Hermitian symmetry of
// the DFT of a real sequence (the inverse takes Re and Im of the packed result).
//
// Planes of side 32..128 always take this path; 256 only with
// DMCR_FLAG_FUSED_PLANES (one plane then holds a whole compute unit, so its loads
// and stores cannot overlap: fewer bytes, but a lower bandwidth than two passes).
//
// Pencil DFTs are those of fft_reg.h: the contiguous-axis rows use the packed
// real transform of length n/2 with lanes along a row; the columns use lanes
// across columns, so every LDS gather and every global store of the column
// phase is a run of adjacent columns.
#include "dmcr_internal.h"
#include "fft_reg.h"

namespace dmcr {

namespace {

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Thread geometry.  A lane set of R2 threads per row (row phases) or per
// column (column phases) covers nb = n/2 / NB rows or columns; with NB = 2 (n =
// 256) each thread runs two lane sets in turn, so that one thread's share of the
// waiting half plane and its pencil registers fit the register file at 8 waves.
template <int L>
struct Plane {
    static constexpr int n = 1 << L;
    static constexpr int nh = n / 2;         // complex row length, rows per half, packed columns
    static constexpr int LH = L - 1;
    using SP = Split<LH>;
    static constexpr int R1 = SP::R1, R2 = SP::R2, S = SP::S;
    static constexpr int NB = L >= 8 ? 2 : 1;
    static constexpr int nb = nh / NB;
    static constexpr int threads = R2 * nb;
    // LDS: one region per lane set, holding its pencil exchange or its share of
    // a staged half plane (columns h nb.. of every row for the forward column
    // phase, rows h nb.. for the inverse row phase), then the packed column.
    // Row pitches of R2 mod 32 float2: the rows that a wave touches at once (R2
    // lanes of 8 bytes each) start R2 * 8 bytes apart in the 64 four-byte banks.
    static constexpr int cpitch = nb + R2;   // forward staging: row pitch within a column set
    static constexpr int rpitch = nh + R2;   // inverse staging and the natural-order rows
    static constexpr int region = cmax(cmax(ex_size<LH>(nb), nh * cpitch), nb * rpitch);
    static constexpr int lds_len = NB * region + nh;
    // the staging index maps use R2 | nb and R1 | nb (a lane set's column or row
    // range starts on a multiple of R2 or R1); the launch uses one block per plane
    static_assert(nb % R2 == 0 && nb % R1 == 0, "lane set must hold whole R1 and R2 groups");
    static_assert(threads <= 1024 && lds_len * 8 <= 160 * 1024, "one plane per workgroup must fit a CU");
};

// threadIdx.x behind an optimisation barrier: the index arithmetic of a phase is
// then done within that phase, instead of being hoisted to the kernel entry and
// kept live next to the half plane that waits in registers.
__device__ __forceinline__ int phase_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Column-phase lanes: c = column within the lane set, q = row set.  With at
// least 64 columns per set q is the same across a wave; saying so keeps the
// row offsets in scalar registers.
template <int NB_COLS>
__device__ __forceinline__ void col_lane(int &c, int &q)
{
    const int tid = phase_tid();
    c = tid % NB_COLS;
    q = tid / NB_COLS;
    if constexpr (NB_COLS >= 64) q = __builtin_amdgcn_readfirstlane(q);
}

// w * W_n^M (forward) or w * W_n^-M (inverse), n = 2^L, M a compile-time constant
template <bool INV, int L, int M>
__device__ __forceinline__ float2 tw_mul_const(float2 w)
{
    if constexpr (M == 0) {
        return w;
    } else {
        constexpr cf c = unit_root(M, 1 << L);
        return c_mul(w, make_float2(c.x, INV ? -c.y : c.y));
    }
}

// The NB pencils of a thread (one per lane set) through one exchange: pencil
// i exchanges in LDS region i; all share lane p's twiddles and the two barriers.
// In: v[i][i1] = x_i[R2 i1 + p].  Out: u[i][s][k2] = X_i[(p + R2 s) + R1 k2].
template <int LH, bool INV, int LO, int NB>
__device__ __forceinline__ void pencils_fwd(float2 (&v)[NB][Split<LH>::R1],
                                            float2 (&u)[NB][Split<LH>::S][Split<LH>::R2], float2 *lds, int region,
                                            int p, int t, int T)
{
    using SP = Split<LH>;
    float2 tw[SP::R1];
    tw_powers<INV>(p, LH, tw);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        dft_reg<SP::R1, INV>(v[i]);
        static_for<0, SP::R1>([&](auto kc) {
            constexpr int k1 = decltype(kc)::value;
            float2 w = v[i][k1];
            if constexpr (k1 != 0) w = c_mul(w, tw[k1]);
            lds[i * region + ex_idx<LH, LO>(k1, p, t, T)] = w;
        });
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i)
        static_for<0, SP::S>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            const int k1 = p + SP::R2 * s;
            static_for<0, SP::R2>([&](auto ic) {
                constexpr int i2 = decltype(ic)::value;
                u[i][s][i2] = lds[i * region + ex_idx<LH, LO>(k1, i2, t, T)];
            });
            dft_reg<SP::R2, INV>(u[i][s]);
        });
    __syncthreads();
}

// Rows h nb + t (h < NB) of a half plane starting at `rows` (rows of nh float2
// pairs): v[h][i1] = row pair R2 i1 + p, lanes p < R2 along a row.
template <int L>
__device__ __forceinline__ void rows_load(const float2 *rows, float2 (&v)[Plane<L>::NB][Plane<L>::R1])
{
    using G = Plane<L>;
    const int tid = phase_tid();
    const int p = tid % G::R2, t = tid / G::R2;
#pragma unroll
    for (int h = 0; h < G::NB; ++h) {
        const float2 *row = rows + (size_t)(h * G::nb + t) * G::nh + p;
#pragma unroll
        for (int i1 = 0; i1 < G::R1; ++i1) v[h][i1] = row[G::R2 * i1];
    }
}

// Contiguous-axis real-to-half transforms of the rows rows_load fetched (the
// next half's loads can be in flight meanwhile).  out[h][j] = X[p + R2 j] of
// row h nb + t for j < R1, except that lane 0 returns X_0 + i X_{n/2} in
// out[h][0].  A whole phase: it ends with a barrier.
template <int L>
__device__ __forceinline__ void rows_r2c(float2 (&v)[Plane<L>::NB][Plane<L>::R1],
                                         float2 (&out)[Plane<L>::NB][Plane<L>::R1], float2 *lds)
{
    using G = Plane<L>;
    constexpr int nh = G::nh, nb = G::nb, NB = G::NB, LH = G::LH, R1 = G::R1, R2 = G::R2, S = G::S,
                  zp = G::rpitch;
    const int tid = phase_tid();
    const int p = tid % R2, t = tid / R2;
    float2 u[NB][S][R2];
    pencils_fwd<LH, false, LANE_P, NB>(v, u, lds, G::region, p, t, nb);
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) lds[h * G::region + t * zp + (p + R2 * s) + R1 * k2] = u[h][s][k2];
    __syncthreads();
    const float2 wp = tw_n<false>(p, L);
#pragma unroll
    for (int h = 0; h < NB; ++h) {
        const float2 *z = lds + h * G::region + t * zp;
        static_for<0, R1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const int k = p + R2 * j;
            const float2 zk = z[k];
            const float2 zc = c_conj(z[(nh - k) & (nh - 1)]);
            const float2 E = c_scale(c_add(zk, zc), 0.5f);
            const float2 d = c_sub(zk, zc);                   // 2i O
            const float2 O = make_float2(0.5f * d.y, -0.5f * d.x);
            out[h][j] = c_add(E, c_mul(O, tw_mul_const<false, L, R2 * j>(wp)));
        });
        if (p == 0) {
            const float2 z0 = z[0];
            out[h][0] = make_float2(z0.x + z0.y, z0.x - z0.y);   // (X_0, X_{n/2}), both real
        }
    }
    __syncthreads();
}

// Axis-1 forward of one half-length column set (rows 2m + PAR of the result).
// val[h][j] = row h nb + t, column p + R2 j of the set (packed column 0).
// Writes the rows to dst (row pitch hp), columns 0 and n/2 separated.
template <int L, int PAR>
__device__ __forceinline__ void col_fwd(const float2 (&val)[Plane<L>::NB][Plane<L>::R1], float2 *lds, float2 *dst,
                                        int hp)
{
    using G = Plane<L>;
    constexpr int nh = G::nh, nb = G::nb, NB = G::NB, LH = G::LH, R1 = G::R1, R2 = G::R2, S = G::S,
                  cp = G::cpitch;
    float2 *cz = lds + NB * G::region;
    {
        const int tid = phase_tid();
        const int p = tid % R2, t = tid / R2;
        // column p + R2 j lies in set (p + R2 j) / nb = R2 j / nb (R2 divides nb)
#pragma unroll
        for (int h = 0; h < NB; ++h)
#pragma unroll
            for (int j = 0; j < R1; ++j) {
                const int hc = (R2 * j) / nb;
                lds[hc * G::region + (h * nb + t) * cp + p + R2 * j - hc * nb] = val[h][j];
            }
    }
    __syncthreads();
    int c, q;
    col_lane<nb>(c, q);
    float2 v[NB][R1];
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
        for (int i1 = 0; i1 < R1; ++i1) v[h][i1] = lds[h * G::region + (R2 * i1 + q) * cp + c];
    __syncthreads();
    float2 u[NB][S][R2];
    pencils_fwd<LH, false, LANE_T, NB>(v, u, lds, G::region, q, c, nb);
    // u[h][s][k2] = Y[m] of column h nb + c, m = (q + R2 s) + R1 k2
    if (c == 0) {
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) cz[(q + R2 * s) + R1 * k2] = u[0][s][k2];
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < NB; ++h) {
        float2 *col = dst + h * nb + c;
        if (h != 0 || c != 0) {
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int m = (q + R2 * s) + R1 * k2;
                    col[(size_t)(2 * m + PAR) * hp] = u[h][s][k2];
                }
        } else {
            // Y = P + i Q with P, Q the transforms of two real sequences: P[m'] =
            // conj P[m] for m' = -m (even rows) or m' = -1 - m (odd rows, twiddled)
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int m = (q + R2 * s) + R1 * k2;
                    const int mp = PAR == 0 ? ((nh - m) & (nh - 1)) : (nh - 1 - m);
                    const float2 y = u[0][s][k2];
                    const float2 yc = c_conj(cz[mp]);
                    const float2 P = c_scale(c_add(y, yc), 0.5f);
                    const float2 D = c_sub(y, yc);
                    const float2 Q = make_float2(0.5f * D.y, -0.5f * D.x);
                    float2 *row = dst + (size_t)(2 * m + PAR) * hp;
                    row[0] = P;
                    row[nh] = Q;
                }
        }
    }
}

// float64 sum of a thread's loaded share of a half plane
template <int L>
__device__ __forceinline__ double rows_sum(const float2 (&v)[Plane<L>::NB][Plane<L>::R1])
{
    double sm = 0.0;
#pragma unroll
    for (int h = 0; h < Plane<L>::NB; ++h)
#pragma unroll
        for (int i1 = 0; i1 < Plane<L>::R1; ++i1) {
            sm += (double)v[h][i1].x;
            sm += (double)v[h][i1].y;
        }
    return sm;
}

// in: real planes [nplanes][n][n]; out: half spectra [nplanes][n][hp].  With
// msum, msum[plane * waves + wave] = float64 sum of the wave's share of the plane.
template <int L>
__global__ __launch_bounds__(Plane<L>::threads) void k_plane_fwd(const float *in, float2 *out, int hp, double *msum)
{
    using G = Plane<L>;
    constexpr int n = G::n, nh = G::nh, nb = G::nb, NB = G::NB, R1 = G::R1, R2 = G::R2;
    __shared__ float2 lds[G::lds_len];
    const int64_t pl = blockIdx.x;
    const float2 *src = reinterpret_cast<const float2 *>(in + pl * n * n);   // row r at src + r nh
    float2 *dst = out + pl * n * hp;
    float2 a[NB][R1], b[NB][R1];
    {
        float2 v[NB][R1], vn[NB][R1];
        rows_load<L>(src, v);
        rows_load<L>(src + (size_t)nh * nh, vn);   // second half in flight during the first
        double sm = msum ? rows_sum<L>(v) : 0.0;
        rows_r2c<L>(v, a, lds);
        if (msum) {
            sm = group_sum(sm + rows_sum<L>(vn), 64);
            const int tid = phase_tid();
            if ((tid & 63) == 0) msum[pl * (G::threads / 64) + tid / 64] = sm;
        }
        rows_r2c<L>(vn, b, lds);
    }
    const int t = phase_tid() / R2;
#pragma unroll
    for (int h = 0; h < NB; ++h) {
        const float2 w = tw_n<false>(h * nb + t, L);
#pragma unroll
        for (int j = 0; j < R1; ++j) {
            const float2 s = c_add(a[h][j], b[h][j]);
            b[h][j] = c_mul(c_sub(a[h][j], b[h][j]), w);
            a[h][j] = s;
        }
    }
    col_fwd<L, 0>(a, lds, dst, hp);
    col_fwd<L, 1>(b, lds, dst, hp);
}

// Contiguous-axis half-to-real transform of the half plane staged from the
// column phase (val[h][s][k2] = row (q + R2 s) + R1 k2, column h nb + c; packed
// column 0).  dst: the real rows as pairs, row r at dst + r nh.  With PRO, each
// output also takes cw times its parent in the coarser plane cplane (rows of nh
// reals; fine row row0 + r has parent row (row0 + r) / 2, and the two reals of
// pair j share the parent j).
template <int L, bool PRO = false>
__device__ __forceinline__ void row_c2r(const float2 (&val)[Plane<L>::NB][Plane<L>::S][Plane<L>::R2], float2 *lds,
                                        float2 *dst, const float *cplane = nullptr, int row0 = 0, float cw = 0.f)
{
    using G = Plane<L>;
    constexpr int nh = G::nh, nb = G::nb, NB = G::NB, LH = G::LH, R1 = G::R1, R2 = G::R2, S = G::S,
                  rp = G::rpitch;
    {
        int c, q;
        col_lane<nb>(c, q);
        // row (q + R2 s) + R1 k2 lies in row set ((q + R2 s) + R1 k2) / nb = R1 k2 / nb
        // (q + R2 s < R1 and R1 divides nb)
#pragma unroll
        for (int h = 0; h < NB; ++h)
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int hr = (R1 * k2) / nb;
                    lds[hr * G::region + ((q + R2 * s) + R1 * k2 - hr * nb) * rp + h * nb + c] = val[h][s][k2];
                }
    }
    __syncthreads();
    const int tid = phase_tid();
    const int p = tid % R2, t = tid / R2;
    const float2 wp = tw_n<true>(p, L);
    float2 v[NB][R1];
#pragma unroll
    for (int h = 0; h < NB; ++h) {
        const float2 *x = lds + h * G::region + t * rp;
        static_for<0, R1>([&](auto ic) {
            constexpr int i1 = decltype(ic)::value;
            const int k = R2 * i1 + p;
            float2 xk = x[k];
            float2 xc = x[(nh - k) & (nh - 1)];
            if constexpr (i1 == 0) {
                if (p == 0) {            // X_0 and X_{n/2} from the packed column
                    xc = make_float2(xk.y, 0.f);
                    xk = make_float2(xk.x, 0.f);
                }
            }
            const float2 xm = c_conj(xc);
            const float2 e = c_add(xk, xm);
            const float2 o = c_mul(c_sub(xk, xm), tw_mul_const<true, L, R2 * i1>(wp));   // W_n^-k (X[k] - conj X[n/2-k])
            v[h][i1] = make_float2(e.x - o.y, e.y + o.x);                                  // e + i o
        });
    }
    __syncthreads();
    float2 u[NB][S][R2];
    pencils_fwd<LH, true, LANE_P, NB>(v, u, lds, G::region, p, t, nb);
#pragma unroll
    for (int h = 0; h < NB; ++h) {
        float2 *row = dst + (size_t)(h * nb + t) * nh;
        if constexpr (PRO) {
            const float *cr = cplane + (size_t)((row0 + h * nb + t) / 2) * nh;
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int j = (p + R2 * s) + R1 * k2;
                    const float c = cr[j];
                    row[j] = make_float2(fmaf(cw, c, u[h][s][k2].x), fmaf(cw, c, u[h][s][k2].y));
                }
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) row[(p + R2 * s) + R1 * k2] = u[h][s][k2];
        }
    }
}

// Loads of the column sets of rows 2m + PAR of a half spectrum (row pitch hp):
// v[h][i1] = row 2 (R2 i1 + q) + PAR, column h nb + c, and y[i1] = column n/2
// of that row (used by the lane of column 0, where columns 0 and n/2 travel
// packed).
template <int L, int PAR>
__device__ __forceinline__ void cols_load(const float2 *src, int hp, float2 (&v)[Plane<L>::NB][Plane<L>::R1],
                                          float2 (&y)[Plane<L>::R1])
{
    using G = Plane<L>;
    constexpr int nh = G::nh, nb = G::nb, R1 = G::R1, R2 = G::R2;
    int c, q;
    col_lane<nb>(c, q);
#pragma unroll
    for (int h = 0; h < G::NB; ++h) {
        const float2 *col = src + h * nb + c;
#pragma unroll
        for (int i1 = 0; i1 < R1; ++i1) v[h][i1] = col[(size_t)(2 * (R2 * i1 + q) + PAR) * hp];
    }
    if (c == 0) {
#pragma unroll
        for (int i1 = 0; i1 < R1; ++i1) y[i1] = src[(size_t)(2 * (R2 * i1 + q) + PAR) * hp + nh];
    }
}

// Axis-1 inverse of the loaded column sets: u[h][s][k2] = row (q + R2 s) + R1 k2
// of the half-length transform of column h nb + c.
template <int L>
__device__ __forceinline__ void cols_inv(float2 (&v)[Plane<L>::NB][Plane<L>::R1], const float2 (&y)[Plane<L>::R1],
                                         float2 (&u)[Plane<L>::NB][Plane<L>::S][Plane<L>::R2], float2 *lds)
{
    using G = Plane<L>;
    constexpr int nb = G::nb, LH = G::LH, R1 = G::R1;
    int c, q;
    col_lane<nb>(c, q);
    if (c == 0) {   // Z = X_0 + i X_{n/2}
#pragma unroll
        for (int i1 = 0; i1 < R1; ++i1) v[0][i1] = make_float2(v[0][i1].x - y[i1].y, v[0][i1].y + y[i1].x);
    }
    pencils_fwd<LH, true, LANE_T, G::NB>(v, u, lds, G::region, q, c, nb);
}

// in: half spectra [nplanes][n][hp]; out: real planes [nplanes][n][n] (both
// axes inverse, unnormalised).  With PRO, plane pl = bc n0 + z also adds cw times
// the coarser level's plane bc n0/2 + z/2 of `coarse` at each voxel's parent.
template <int L, bool PRO>
__global__ __launch_bounds__(Plane<L>::threads) void k_plane_inv(const float2 *in, float *out, int hp,
                                                                 const float *coarse, float cw, int n0)
{
    using G = Plane<L>;
    constexpr int n = G::n, nh = G::nh, nb = G::nb, NB = G::NB, R1 = G::R1, R2 = G::R2, S = G::S;
    __shared__ float2 lds[G::lds_len];
    const int64_t pl = blockIdx.x;
    const float2 *src = in + pl * n * hp;
    float2 *dst = reinterpret_cast<float2 *>(out + pl * n * n);
    float2 se[NB][S][R2], so[NB][S][R2];
    {
        float2 v[NB][R1], y[R1], vn[NB][R1], yn[R1];
        cols_load<L, 0>(src, hp, v, y);
        cols_load<L, 1>(src, hp, vn, yn);   // odd rows in flight during the even ones
        cols_inv<L>(v, y, se, lds);
        cols_inv<L>(vn, yn, so, lds);
    }
    int c, q;
    col_lane<nb>(c, q);
    // rows r and r + n/2, r = (q + R2 s) + R1 k2: se[r] +- W_n^-r so[r]
    static_for<0, S>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        const float2 wb = tw_n<true>(q + R2 * s, L);
        static_for<0, R2>([&](auto kc) {
            constexpr int k2 = decltype(kc)::value;
            const float2 w = tw_mul_const<true, L, R1 * k2>(wb);
#pragma unroll
            for (int h = 0; h < NB; ++h) {
                const float2 o = c_mul(so[h][s][k2], w);
                so[h][s][k2] = c_sub(se[h][s][k2], o);
                se[h][s][k2] = c_add(se[h][s][k2], o);
            }
        });
    });
    if constexpr (PRO) {
        const int64_t bc = pl / n0, z = pl % n0;
        const float *cplane = coarse + (bc * (n0 / 2) + z / 2) * nh * nh;
        row_c2r<L, true>(se, lds, dst, cplane, 0, cw);
        row_c2r<L, true>(so, lds, dst + (size_t)nh * nh, cplane, nh, cw);
    } else {
        row_c2r<L>(se, lds, dst);
        row_c2r<L>(so, lds, dst + (size_t)nh * nh);
    }
}

// the prolongation of the inverse (coarse, cw, n0) is used when coarse is set;
// msum: the forward's partial sums of the means (or null)
struct PlanePro {
    const float *coarse;
    float cw;
    int n0;
    double *msum;
};

template <int L>
hipError_t plane_launch(bool inv, const void *in, void *out, int64_t nplanes, int hp, double bytes, hipStream_t st,
                        PlanePro pro)
{
    const dim3 g((unsigned)nplanes), b(Plane<L>::threads);
    if (inv && pro.coarse)
        return launch("plane_inv", bytes, k_plane_inv<L, true>, g, b, 0, st, static_cast<const float2 *>(in),
                      static_cast<float *>(out), hp, pro.coarse, pro.cw, pro.n0);
    if (inv)
        return launch("plane_inv", bytes, k_plane_inv<L, false>, g, b, 0, st, static_cast<const float2 *>(in),
                      static_cast<float *>(out), hp, (const float *)nullptr, 0.f, 1);
    return launch("plane_fwd", bytes, k_plane_fwd<L>, g, b, 0, st, static_cast<const float *>(in),
                  static_cast<float2 *>(out), hp, pro.msum);
}

hipError_t plane_dispatch(bool inv, int L, const void *in, void *out, int64_t nplanes, int hp, double bytes,
                          hipStream_t st, PlanePro pro = PlanePro{nullptr, 0.f, 1, nullptr})
{
    switch (L) {
    case 5: return plane_launch<5>(inv, in, out, nplanes, hp, bytes, st, pro);
    case 6: return plane_launch<6>(inv, in, out, nplanes, hp, bytes, st, pro);
    case 7: return plane_launch<7>(inv, in, out, nplanes, hp, bytes, st, pro);
    case 8: return plane_launch<8>(inv, in, out, nplanes, hp, bytes, st, pro);
    }
    return hipErrorInvalidValue;
}

int plane_log2(const LevelPlan &L)
{
    int l = 0;
    while ((1 << l) < L.n[1]) ++l;
    return l;
}

}  // namespace

bool plane_supported(const Plan &p, int l)
{
    if (p.ndim != 3) return false;
    const LevelPlan &L = p.lv[l];
    if (L.n[1] != L.n[2]) return false;
    const int lg = plane_log2(L);
    if (lg == 8 && !(p.flags & DMCR_FLAG_FUSED_PLANES)) return false;
    return lg >= 5 && lg <= 8 && L.h == L.n[2] / 2 + 1;
}

int plane_waves(const Plan &p, int l)
{
    switch (plane_log2(p.lv[l])) {
    case 5: return Plane<5>::threads / 64;
    case 6: return Plane<6>::threads / 64;
    case 7: return Plane<7>::threads / 64;
    default: return Plane<8>::threads / 64;
    }
}

hipError_t plane_forward(const Plan &p, int l, const float *phi, float2 *X, hipStream_t st, double *msum)
{
    const LevelPlan &L = p.lv[l];
    if (!plane_supported(p, l)) return hipErrorInvalidValue;
    const int64_t nplanes = (int64_t)p.B * p.C * L.n[0];
    if (nplanes >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    const double bytes = (double)nplanes * L.n[1] * ((double)L.n[2] * 4 + (double)L.h * 8);
    return plane_dispatch(false, plane_log2(L), phi, X, nplanes, L.hp, bytes, st, PlanePro{nullptr, 0.f, 1, msum});
}

hipError_t plane_inverse(const Plan &p, int l, const float2 *X, float *grad, hipStream_t st, const float *coarse)
{
    const LevelPlan &L = p.lv[l];
    if (!plane_supported(p, l)) return hipErrorInvalidValue;
    const int64_t nplanes = (int64_t)p.B * p.C * L.n[0];
    if (nplanes >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    if (coarse && L.n[0] % 2) return hipErrorInvalidValue;
    double bytes = (double)nplanes * L.n[1] * ((double)L.n[2] * 4 + (double)L.h * 8);
    if (coarse) bytes += (double)nplanes * L.n[1] * L.n[2] * 4 / 8;   // the coarse level: 1/8 of the voxels
    return plane_dispatch(true, plane_log2(L), X, grad, nplanes, L.hp, bytes, st,
                          PlanePro{coarse, 0.125f, L.n[0], nullptr});
}

}  // namespace dmcr
