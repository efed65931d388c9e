// Three-point correlations of each channel (Sec. 3.2.2, eq. s3) over the
// unordered pairs of a small displacement box, their adjoint, and the Appendix A
// map of the soft-threshold form (eq. s3rfroms3rbar).
//
// With the M vectors r_c of [-P3, P3]^d, a block of voxels builds in LDS the
// realisations E[x][c]: soft threshold E = f((phi(x) + phi(x + r_c)) / 2);
// product form E = phi(x + r_c) with the weight w(x) = phi(x).  The block's
// share of S3(a, b) is sum_x w(x) E[x][a] E[x][b] (w = 1 for the soft form), a
// small dense Gram product; block partials are added in float64, in block order.
// Adjoint, with Ghat the symmetric M x M cotangent (diagonal doubled) and
// D[x][c] = (1/N) sum_d Ghat(c, d) E[x][d]:
//   soft:    Q_c(x) = f'(u_c(x)) D[x][c] / 2,   grad(y) += sum_c Q_c(y) + sum_c Q_c(y - r_c)
//   product: Q_c(x) = w(x) D[x][c],  R_c(x) = E[x][c] D[x][c] / 2,
//            grad(y) += sum_c R_c(y) + sum_c Q_c(y - r_c)
// (the first sum is the start point x = y, the second the end point y = x + r_c).
// Both contractions run on the FP32 matrix cores (v_mfma_f32_16x16x4f32) where
// the level allows it (below); otherwise register-blocked, each thread owning a
// 4 x 4 output tile and reading two float4 per 16 multiply-adds.
//
// Matrix-core forward: a block loads its box of voxels with a halo of P3 into
// LDS; a realisation is one LDS read at the voxel's tile address plus the
// offset of r_c (the soft threshold applied on the fly).  The Gram matrix is cut
// into 16 x 16 tiles; a wave owns a super-tile of 6 x 6 of them (on the
// diagonal only the upper triangle) and the four waves of the block split the
// box's voxels, four per instruction; their accumulators are added in LDS in
// wave order.  Matrix-core adjoint: D = E Gf / N for 64 voxels x 96 vectors per
// wave and pass (16 tiles of 16 x 16, K = 4 vectors d per instruction), then Q
// is stored and the local term (R for the product form, Q_c(y) for the soft
// one) is summed over c in registers and added to the gradient directly, so
// only the shifted sum sum_c Q_c(y - r_c) is left to the gather.
#include <algorithm>

#include "dmcr_internal.h"
#include "fft_reg.h"

namespace dmcr {

namespace {

constexpr int kT3 = 256;
constexpr size_t kS3Lds = 60 * 1024;

struct S3Geo {
    int ndim, n0, n1, n2;
    int64_t N;
    int P3, box, M;
    int64_t K3;
};

// soft threshold of the pair mean (a + b) / 2, its exponent's constants folded:
// exp(-alpha ((a + b) / 2 + c2)) = 2^(k1 (a + b) + k0), k1 = -alpha log2(e) / 2,
// k0 = -alpha c2 log2(e)
struct SoftC {
    float alpha, c1, c2, c3, k1, k0;
};

// sigma((a + b) / 2) = 1 / (1 + 2^(k1 (a + b) + k0)), given s = a + b
__device__ __forceinline__ float soft_sig(float s, const SoftC &c)
{
    return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(fmaf(s, c.k1, c.k0)));
}

__device__ __forceinline__ void vec_of(const S3Geo &g, int v, int &c0, int &c1, int &c2)
{
    if (g.ndim == 2) {
        c0 = v / g.box - g.P3;
        c1 = v % g.box - g.P3;
        c2 = 0;
    } else {
        c2 = v % g.box - g.P3;
        c1 = (v / g.box) % g.box - g.P3;
        c0 = v / (g.box * g.box) - g.P3;
    }
}

// voxel x + (c0, c1, c2), periodic (every axis a power of two)
__device__ __forceinline__ int64_t shift(const S3Geo &g, int64_t x, int c0, int c1, int c2)
{
    const int i2 = (int)(x % g.n2);
    const int i1 = (int)((x / g.n2) % g.n1);
    const int i0 = (int)(x / ((int64_t)g.n1 * g.n2));
    return ((int64_t)((i0 + c0) & (g.n0 - 1)) * g.n1 + ((i1 + c1) & (g.n1 - 1))) * g.n2 + ((i2 + c2) & (g.n2 - 1));
}

// first entry of row a of the upper triangle (r_a-major order)
__device__ __forceinline__ int64_t tri_row(int a, int M) { return (int64_t)a * M - (int64_t)a * (a - 1) / 2; }

__device__ __forceinline__ void tri_decode(int64_t k, int M, int &a, int &b)
{
    int lo = 0, hi = M - 1;   // largest a with tri_row(a) <= k
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (tri_row(mid, M) <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    a = lo;
    b = a + (int)(k - tri_row(a, M));
}

// Realisation of vector c at voxel x (soft: f(u_c(x)); product: phi(x + r_c)).
template <bool SOFT>
__device__ __forceinline__ float realisation(const S3Geo &g, const float *__restrict__ f, int64_t x, int c,
                                             const SoftC &sc)
{
    int c0, c1, c2;
    vec_of(g, c, c0, c1, c2);
    const float fy = f[shift(g, x, c0, c1, c2)];
    if constexpr (SOFT)
        return fmaf(sc.c1, soft_sig(f[x] + fy, sc), sc.c3);
    else
        return fy;
}

struct S3FwdArgs {
    S3Geo g;
    SoftC sc;
    const float *phi;   // level field [B][C][N]
    float *part;        // [B][C][chunks][K3]
    int C, VB, Mp;      // Mp = M rounded up to 4 (zero columns)
    int64_t chunks;
};

// Block partial of S3: E[xl][0..Mp) rows in LDS; thread t owns the 4 x 4 tile
// (rows a0..a0+3, columns b0..b0+3) of E^T diag(w) E for tile pairs b0 >= a0.
template <bool SOFT>
__global__ __launch_bounds__(kT3) void k_s3_fwd(S3FwdArgs a)
{
    extern __shared__ float4 sm4[];
    const S3Geo &g = a.g;
    const int64_t chunk = blockIdx.x;
    const int ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    const int Mp = a.Mp, M = g.M;
    float *E = reinterpret_cast<float *>(sm4);
    float *w = E + a.VB * Mp;
    const float *f = a.phi + (b * a.C + ch) * g.N;
    const int64_t x0 = chunk * a.VB;
    for (int idx = threadIdx.x; idx < a.VB * Mp; idx += kT3) {
        const int xl = idx / Mp, c = idx % Mp;
        E[idx] = c < M ? realisation<SOFT>(g, f, x0 + xl, c, a.sc) : 0.f;
    }
    for (int xl = threadIdx.x; xl < a.VB; xl += kT3) w[xl] = SOFT ? 1.f : f[x0 + xl];
    __syncthreads();
    float *out = a.part + ((b * a.C + ch) * a.chunks + chunk) * g.K3;
    const int nb = Mp / 4;
    const int ntiles = nb * (nb + 1) / 2;
    for (int t = threadIdx.x; t < ntiles; t += kT3) {
        // tile t -> (ta, tb), tb >= ta, ta-major
        int ta = 0, rem = t;
        while (rem >= nb - ta) {
            rem -= nb - ta;
            ++ta;
        }
        const int tb = ta + rem;
        float acc[4][4] = {};
        for (int xl = 0; xl < a.VB; ++xl) {
            const float4 ea = *reinterpret_cast<const float4 *>(E + xl * Mp + 4 * ta);
            const float4 eb = *reinterpret_cast<const float4 *>(E + xl * Mp + 4 * tb);
            const float wx = w[xl];
            const float av[4] = {ea.x * wx, ea.y * wx, ea.z * wx, ea.w * wx};
            const float bv[4] = {eb.x, eb.y, eb.z, eb.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(av[i], bv[j], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ia = 4 * ta + i, ib = 4 * tb + j;
                if (ia <= ib && ib < M) out[tri_row(ia, M) + (ib - ia)] = acc[i][j];
            }
    }
}

struct S3RedArgs {
    const float *part;
    float *S;
    int C;
    int64_t chunks, K3, Kstride, off;
    double invN;
};

// one block per (32 consecutive entries, channel, field); lane group q of 8 adds
// chunks q, q + 8, ... in order, then the 8 group sums are added in group order
constexpr int kRK = 32, kRG = kT3 / kRK;

__global__ __launch_bounds__(kT3) void k_s3_reduce(S3RedArgs a)
{
    __shared__ double red[kRG][kRK];
    const int kk = threadIdx.x % kRK, grp = threadIdx.x / kRK;
    const int64_t k = (int64_t)blockIdx.x * kRK + kk;
    const int ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    double s = 0.0;
    if (k < a.K3) {
        const float *src = a.part + (b * a.C + ch) * a.chunks * a.K3 + k;
        for (int64_t t = grp; t < a.chunks; t += kRG) s += (double)src[t * a.K3];
    }
    red[grp][kk] = s;
    __syncthreads();
    if (grp == 0 && k < a.K3) {
        double tot = red[0][kk];
        for (int q = 1; q < kRG; ++q) tot += red[q][kk];
        a.S[b * a.Kstride + a.off + ch * a.K3 + k] = (float)(tot * a.invN);
    }
}

// cotangent entry i of the packed descriptor-shaped G; with St, G holds the
// descriptor S and the entry is 2 w^2 (S - St) / Z, in float64 in the error
// kernel's order, so it has the error kernel's bits
__device__ __forceinline__ float s3_cot(const float *G, const double *St, double w2, double invZ, int64_t i)
{
    if (!St) return G[i];
    const double d = (double)G[i] - St[i];
    return (float)(2.0 * w2 * d * invZ);
}

struct S3AdjArgs {
    S3Geo g;
    SoftC sc;
    const float *phi;
    const float *G;     // cotangent [B][Kstride]; with St: the descriptor S
    const double *St;   // target descriptor [B][Kstride], or null
    double w2, invZ;    // with St: the level's w_l^2 and 1 / Z
    float *Gf;          // [B][C][M][Mp] full symmetric cotangent, diagonal doubled
    float *Q, *R;       // [B][C][M][N]
    float *grad;        // level gradient [B][C][N] (added to)
    int C, VB, Mp, Kp;
    int64_t Kstride, off;
    float invN;
};

// Gf[c][d] = G(min, max), doubled on the diagonal, zero in the padding rows
// (c >= M, up to Kp) and columns (d >= M, up to Mp)
__global__ __launch_bounds__(kT3) void k_s3_expand(S3AdjArgs a)
{
    const S3Geo &g = a.g;
    const int ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    const int64_t gb = b * a.Kstride + a.off + ch * g.K3;
    float *out = a.Gf + (b * a.C + ch) * (int64_t)a.Kp * a.Mp;
    for (int64_t idx = (int64_t)blockIdx.x * kT3 + threadIdx.x; idx < (int64_t)a.Kp * a.Mp;
         idx += (int64_t)gridDim.x * kT3) {
        const int c = (int)(idx / a.Mp), d = (int)(idx % a.Mp);
        float v = 0.f;
        if (c < g.M && d < g.M) {
            const int lo = c < d ? c : d, hi = c < d ? d : c;
            v = s3_cot(a.G, a.St, a.w2, a.invZ, gb + tri_row(lo, g.M) + (hi - lo)) * (c == d ? 2.f : 1.f);
        }
        out[idx] = v;
    }
}

// D = E Gf / N for VB voxels: Et[d][xl] (transposed realisations) in LDS, Gf rows
// read as float4 (cached); thread tile 4 voxels x 4 vectors; then Q (and R).
template <bool SOFT>
__global__ __launch_bounds__(kT3) void k_s3_adj_terms(S3AdjArgs a)
{
    extern __shared__ float4 sm4[];
    const S3Geo &g = a.g;
    const int64_t chunk = blockIdx.x;
    const int ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    const int M = g.M, Mp = a.Mp, VB = a.VB;
    float *Et = reinterpret_cast<float *>(sm4);   // [M][VB]
    const float *f = a.phi + (b * a.C + ch) * g.N;
    const float *Gf = a.Gf + (b * a.C + ch) * (int64_t)M * Mp;
    const int64_t x0 = chunk * VB;
    for (int idx = threadIdx.x; idx < VB * M; idx += kT3) {
        const int c = idx / VB, xl = idx % VB;
        Et[idx] = realisation<SOFT>(g, f, x0 + xl, c, a.sc);
    }
    __syncthreads();
    const int64_t qbase = (b * a.C + ch) * M;
    const int nx = VB / 4, nc = Mp / 4;
    for (int t = threadIdx.x; t < nx * nc; t += kT3) {
        const int tx = t % nx, tc = t / nx;
        float acc[4][4] = {};
        for (int d = 0; d < M; ++d) {
            const float4 ex = *reinterpret_cast<const float4 *>(Et + d * VB + 4 * tx);
            const float4 gv = *reinterpret_cast<const float4 *>(Gf + (int64_t)d * Mp + 4 * tc);
            const float xv[4] = {ex.x, ex.y, ex.z, ex.w};
            const float cv[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(xv[i], cv[j], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int xl = 4 * tx + i;
            const int64_t x = x0 + xl;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * tc + j;
                if (c >= M) continue;
                const float D = acc[i][j] * a.invN;
                if constexpr (SOFT) {
                    int c0, c1, c2;
                    vec_of(g, c, c0, c1, c2);
                    const float sg = soft_sig(f[x] + f[shift(g, x, c0, c1, c2)], a.sc);
                    a.Q[(qbase + c) * g.N + x] = 0.5f * (a.sc.c1 * a.sc.alpha) * sg * (1.f - sg) * D;
                } else {
                    a.Q[(qbase + c) * g.N + x] = f[x] * D;
                    a.R[(qbase + c) * g.N + x] = 0.5f * Et[c * VB + xl] * D;
                }
            }
        }
    }
}

template <bool SOFT>
__global__ __launch_bounds__(kT3) void k_s3_adj_gather(S3AdjArgs a)
{
    const S3Geo &g = a.g;
    const int64_t y = (int64_t)blockIdx.x * kT3 + threadIdx.x;
    const int ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    if (y >= g.N) return;
    const int64_t qbase = (b * a.C + ch) * g.M;
    float acc = 0.f;
    for (int c = 0; c < g.M; ++c) {
        int c0, c1, c2;
        vec_of(g, c, c0, c1, c2);
        const float *Qc = a.Q + (qbase + c) * g.N;
        acc += Qc[shift(g, y, -c0, -c1, -c2)];
        acc += SOFT ? Qc[y] : a.R[(qbase + c) * g.N + y];
    }
    a.grad[(b * a.C + ch) * g.N + y] += acc;
}

// ---- Appendix A map of the three-point blocks (STILDE) -----------------------
struct S3MapArgs {
    float *S;           // [B][Kstride]: descriptor (forward) or cotangent (adjoint)
    int ndim, C;
    int64_t Kstride;
    double h;           // f(1/2)
    int P3[kMaxLevels], M[kMaxLevels], P[kMaxLevels];
    int64_t K3[kMaxLevels], off3[kMaxLevels];
    int64_t off2[kMaxLevels][kMaxChannels];   // offset of the auto pair (c, c)
    int64_t cnt2[kMaxLevels];                 // its half-box entries
};

__device__ __forceinline__ void vec3(int ndim, int P3, int v, int r[3])
{
    const int box = 2 * P3 + 1;
    if (ndim == 2) {
        r[0] = v / box - P3;
        r[1] = v % box - P3;
        r[2] = 0;
    } else {
        r[2] = v % box - P3;
        r[1] = (v / box) % box - P3;
        r[0] = v / (box * box) - P3;
    }
}

// half-box entry of S2(r) (point symmetry maps r to -r when r is not in the half box)
__device__ __forceinline__ int64_t half_index(int ndim, int P, const int r[3])
{
    const int box = 2 * P + 1;
    int64_t bi = (int64_t)(r[0] + P) * box + (r[1] + P);
    int64_t vol = (int64_t)box * box;
    if (ndim == 3) {
        bi = bi * box + (r[2] + P);
        vol *= box;
    }
    const int64_t center = (vol - 1) / 2;
    return bi >= center ? bi - center : (vol - 1 - bi) - center;
}

// For entry (ia, ib): the S2 indices it reads and their coefficients, and the
// coefficient of Sbar3 itself.  Returns the number of S2 terms.
__device__ __forceinline__ int s3_map_terms(const S3MapArgs &a, int l, int ch, int ia, int ib, int64_t idx[4],
                                            double coef[4], double &cb)
{
    int ra[3], rb[3], d[3] = {0, 0, 0}, z[3] = {0, 0, 0};
    vec3(a.ndim, a.P3[l], ia, ra);
    vec3(a.ndim, a.P3[l], ib, rb);
    const bool za = ra[0] == 0 && ra[1] == 0 && ra[2] == 0;
    const bool zb = rb[0] == 0 && rb[1] == 0 && rb[2] == 0;
    const int64_t o2 = a.off2[l][ch];
    if (ia == ib || zb) {
        cb = 0.0;
        idx[0] = o2 + half_index(a.ndim, a.P[l], ra);
        coef[0] = 1.0;
        return 1;
    }
    if (za) {
        cb = 0.0;
        idx[0] = o2 + half_index(a.ndim, a.P[l], rb);
        coef[0] = 1.0;
        return 1;
    }
    const double q = 1.0 / (1.0 - 2.0 * a.h);
    for (int t = 0; t < 3; ++t) d[t] = ra[t] - rb[t];
    cb = q;
    idx[0] = o2 + half_index(a.ndim, a.P[l], ra);
    idx[1] = o2 + half_index(a.ndim, a.P[l], rb);
    idx[2] = o2 + half_index(a.ndim, a.P[l], z);
    idx[3] = o2 + half_index(a.ndim, a.P[l], d);
    coef[0] = coef[1] = (-a.h + a.h * a.h) * q;
    coef[2] = coef[3] = -a.h * a.h * q;
    return 4;
}

__global__ __launch_bounds__(kT3) void k_s3_map(S3MapArgs a)
{
    const int l = blockIdx.x, ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    float *S = a.S + b * a.Kstride;
    float *S3 = S + a.off3[l] + ch * a.K3[l];
    for (int64_t k = threadIdx.x; k < a.K3[l]; k += kT3) {
        int ia, ib;
        tri_decode(k, a.M[l], ia, ib);
        int64_t idx[4];
        double coef[4], cb;
        const int nt = s3_map_terms(a, l, ch, ia, ib, idx, coef, cb);
        double v = cb * (double)S3[k];
        for (int t = 0; t < nt; ++t) v += coef[t] * (double)S[idx[t]];
        S3[k] = (float)v;
    }
}

// transpose, part 1: every two-point entry of the auto pair (c, c) collects the
// coefficient times the cotangent of each three-point entry whose map reads it
__global__ __launch_bounds__(kT3) void k_s3_map_adj_gather(S3MapArgs a)
{
    const int l = blockIdx.x, ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    float *G = a.S + b * a.Kstride;
    const float *G3 = G + a.off3[l] + ch * a.K3[l];
    for (int64_t h = threadIdx.x; h < a.cnt2[l]; h += kT3) {
        const int64_t me = a.off2[l][ch] + h;
        double acc = 0.0;
        int64_t k = 0;
        for (int ia = 0; ia < a.M[l]; ++ia)
            for (int ib = ia; ib < a.M[l]; ++ib, ++k) {
                int64_t idx[4];
                double coef[4], cb;
                const int nt = s3_map_terms(a, l, ch, ia, ib, idx, coef, cb);
                for (int t = 0; t < nt; ++t)
                    if (idx[t] == me) acc += coef[t] * (double)G3[k];
            }
        G[me] = (float)((double)G[me] + acc);
    }
}

// transpose, part 2: the three-point cotangents scale by their Sbar3 coefficient
__global__ __launch_bounds__(kT3) void k_s3_map_adj_scale(S3MapArgs a)
{
    const int l = blockIdx.x, ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    float *G3 = a.S + b * a.Kstride + a.off3[l] + ch * a.K3[l];
    for (int64_t k = threadIdx.x; k < a.K3[l]; k += kT3) {
        int ia, ib;
        tri_decode(k, a.M[l], ia, ib);
        int64_t idx[4];
        double coef[4], cb;
        s3_map_terms(a, l, ch, ia, ib, idx, coef, cb);
        G3[k] = (float)(cb * (double)G3[k]);
    }
}

// ---- matrix-core contractions ------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kSup = 6;            // 16-wide vector tiles per super-tile side
constexpr int kMfLds = 64 * 1024;  // dynamic LDS limit of one block

struct S3MfArgs {
    S3Geo g;
    SoftC sc;
    const float *phi;   // level field [B][C][N]
    float *part;        // forward: [B][C][chunks][K3]
    const float *Gf;    // adjoint: [B][C][Kp][Mp] expanded cotangent (when it is not built in LDS)
    const float *G;     // adjoint: packed cotangent [B][Kstride], the block at off + channel K3
                        // (with St: the descriptor S, the cotangent formed while reading)
    const double *St;
    double w2, invZ;
    int64_t Kstride, off;
    float *Q;           // adjoint: [B][C][M][N]
    float *grad;        // adjoint: level gradient [B][C][N] (added to)
    int C;
    int bd[3], lb[3];   // voxel box edge per axis and its log2
    int nb[3];          // boxes per axis
    int hl[3];          // halo per axis (P3 on the field's axes, 0 on the unit axis of 2-D)
    int ed[3];          // LDS tile edge per axis, bd + 2 hl
    int64_t chunks;     // boxes per field
    int VB;             // voxels per box
    int n16;            // 16-wide vector tiles on the matrix cores: ceil(M / 16), or M / 16 with rem
    int rem;            // 1: M = 16 n16 + 1, and vector M - 1 (its Gram column and the
                        // adjoint's column of D) is summed by plain FMAs beside the products
    int nst;            // super-tile bands, ceil(n16 / kSup)
    int Kp, Mp;         // rows (M rounded up to 4) and columns (16 ceil(M / 16)) of Gf
    int gs;             // row stride of Gf's copy in LDS (16 mod 32: the four rows of a read hit disjoint banks)
    float invN;
    FastDivU fd_rl, fd_e1, fd_mp;   // exact division by the tile row length, ed[1] and Mp
};

// LDS tile offset of displacement r_c
__device__ __forceinline__ int mf_off(const S3MfArgs &a, int c)
{
    int c0, c1, c2;
    vec_of(a.g, c, c0, c1, c2);
    return (c0 * a.ed[1] + c1) * a.ed[2] + c2;
}

// box coordinates of box voxel v (box edges are powers of two)
__device__ __forceinline__ void mf_coords(const S3MfArgs &a, int v, int &k0, int &k1, int &k2)
{
    k2 = v & (a.bd[2] - 1);
    k1 = (v >> a.lb[2]) & (a.bd[1] - 1);
    k0 = v >> (a.lb[1] + a.lb[2]);
}

// LDS tile address of box voxel v
__device__ __forceinline__ int mf_base(const S3MfArgs &a, int v)
{
    int k0, k1, k2;
    mf_coords(a, v, k0, k1, k2);
    return ((k0 + a.hl[0]) * a.ed[1] + (k1 + a.hl[1])) * a.ed[2] + (k2 + a.hl[2]);
}

// field index of box voxel v of box `chunk`
__device__ __forceinline__ int64_t mf_voxel(const S3MfArgs &a, int64_t chunk, int v)
{
    int k0, k1, k2;
    mf_coords(a, v, k0, k1, k2);
    const int64_t q2 = chunk % a.nb[2], q = chunk / a.nb[2];
    const int64_t q1 = q % a.nb[1], q0 = q / a.nb[1];
    return ((q0 * a.bd[0] + k0) * a.g.n1 + (q1 * a.bd[1] + k1)) * a.g.n2 + (q2 * a.bd[2] + k2);
}

// the box `chunk` of field f with its periodic halo into T, and the zero cell
// T[tv]; each thread issues eight loads before it stores them, so that a block's
// load latency is paid a few times rather than once per element
__device__ __forceinline__ void mf_load_tile(const S3MfArgs &a, const float *__restrict__ f, int64_t chunk, float *T)
{
    constexpr int U = 8;
    const S3Geo &g = a.g;
    const int64_t q2 = chunk % a.nb[2], q = chunk / a.nb[2];
    const int o2 = (int)(q2 * a.bd[2]) - a.hl[2];
    const int o1 = (int)((q % a.nb[1]) * a.bd[1]) - a.hl[1];
    const int o0 = (int)((q / a.nb[1]) * a.bd[0]) - a.hl[0];
    const bool three = g.ndim == 3;
    const int rl = three ? a.ed[2] : a.ed[1];     // row length of the innermost axis
    const int tv = a.ed[0] * a.ed[1] * a.ed[2];
    for (int base = threadIdx.x; base < tv; base += U * blockDim.x) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            v[u] = 0.f;
            if (idx < tv) {
                const int row = fdivu(idx, a.fd_rl), t = idx - row * rl;
                const int t0 = three ? fdivu(row, a.fd_e1) : row;
                const int t1 = three ? row - t0 * a.ed[1] : 0;
                const int64_t rbase = three ? ((int64_t)((o0 + t0) & (g.n0 - 1)) * g.n1 + ((o1 + t1) & (g.n1 - 1))) * g.n2
                                            : (int64_t)((o0 + t0) & (g.n0 - 1)) * g.n1;
                v[u] = f[rbase + (((three ? o2 : o1) + t) & ((three ? g.n2 : g.n1) - 1))];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < tv) T[idx] = v[u];
        }
    }
    if (threadIdx.x == 0) T[tv] = 0.f;   // read in place of the padding vectors past M
}

// realisation from the raw tile values phi(x) and phi(x + r_c); m = 1 for a
// vector of the box, 0 for the padding past M (whose phi(x + r_c) is read from
// the zero cell)
template <bool SOFT>
__device__ __forceinline__ float mf_real(float fx, float fy, float m, const SoftC &sc)
{
    if constexpr (SOFT)
        return m * fmaf(sc.c1, soft_sig(fx + fy, sc), sc.c3);
    else
        return fy;
}

// One super-tile of the forward: NA row tiles from ta0, NB column tiles from tb0
// (DIAG: the same tiles, upper triangle).  The four waves take a quarter of the
// box's voxels each, four per instruction.  A step reads the raw tile values of
// the next four voxels (padding lanes read the zero cell) and then runs the
// current products, so the reads complete under them; then the accumulators of
// the waves are added in LDS in wave order and wave 3 writes the block's
// partial Gram entries.
//
// REM (diagonal super-tiles when M = 16 n16 + 1): each lane also sums
// w(x) E[x][a] E[x][M-1] for its rows a, and w(x) E[x][M-1]^2, by FMAs on the
// A operands it already holds; the Gram column of vector M - 1 then needs no
// 16-wide tile of its own.
template <bool SOFT, bool DIAG, int NA, int NB, bool REM = false>
__device__ __forceinline__ void fwd_super(const S3MfArgs &a, const float *T, f4 *red, int ta0, int tb0, float *out)
{
    static_assert(!REM || DIAG, "the remainder column rides on the diagonal super-tiles");
    const S3Geo &g = a.g;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int zero = a.ed[0] * a.ed[1] * a.ed[2];
    const int offR = REM ? mf_off(a, g.M - 1) : 0;
    float cacc[NA + 1];   // REM: rows of the band against vector M - 1, then the corner
#pragma unroll
    for (int i = 0; i <= NA; ++i) cacc[i] = 0.f;
    int offA[NA], offB[NB];
    bool okA[NA], okB[NB];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int c = 16 * (ta0 + i) + (lane & 15);
        okA[i] = c < g.M;
        offA[i] = okA[i] ? mf_off(a, c) : 0;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int c = 16 * (tb0 + j) + (lane & 15);
        okB[j] = c < g.M;
        offB[j] = okB[j] ? mf_off(a, c) : 0;
    }
    f4 acc[NA][NB];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    // A[i][k] = w(x_k) E[x_k][row i], B[k][j] = E[x_k][column j]: the lane supplies
    // row/column (lane & 15) of voxel k = lane >> 4 of each group of four
    const int vw = a.VB / 4, steps = vw / 4;
    const int v0 = wave * vw + (lane >> 4);
    float fx, yr, ya[NA], yb[NB];   // raw phi(x), phi(x + r_(M-1)), phi(x + r_a), phi(x + r_b)
    auto fetch = [&](int v, float &fx_, float &yr_, float (&ya_)[NA], float (&yb_)[NB]) {
        const int base = mf_base(a, v);
        fx_ = T[base];
        if constexpr (REM) yr_ = T[base + offR];
#pragma unroll
        for (int i = 0; i < NA; ++i) ya_[i] = T[okA[i] ? base + offA[i] : zero];
        if constexpr (!DIAG) {
#pragma unroll
            for (int j = 0; j < NB; ++j) yb_[j] = T[okB[j] ? base + offB[j] : zero];
        }
    };
    fetch(v0, fx, yr, ya, yb);
    for (int s = 0; s < steps; ++s) {
        // the last step reads its own voxels again: no branch around the reads
        float fxn, yrn, yan[NA], ybn[NB];
        fetch(v0 + 4 * min(s + 1, steps - 1), fxn, yrn, yan, ybn);
        __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the products
        const float w = SOFT ? 1.f : fx;
        float ea[NA], eb[NB];
#pragma unroll
        for (int i = 0; i < NA; ++i) ea[i] = mf_real<SOFT>(fx, ya[i], okA[i] ? 1.f : 0.f, a.sc);
        if constexpr (!DIAG) {
#pragma unroll
            for (int j = 0; j < NB; ++j) eb[j] = mf_real<SOFT>(fx, yb[j], okB[j] ? 1.f : 0.f, a.sc);
        }
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const float av = w * ea[i];
#pragma unroll
            for (int j = DIAG ? i : 0; j < NB; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, DIAG ? ea[j] : eb[j], acc[i][j], 0, 0, 0);
        }
        if constexpr (REM) {
            const float er = mf_real<SOFT>(fx, yr, 1.f, a.sc);
#pragma unroll
            for (int i = 0; i < NA; ++i) cacc[i] = fmaf(w * ea[i], er, cacc[i]);
            cacc[NA] = fmaf(w * er, er, cacc[NA]);
        }
        __builtin_amdgcn_sched_barrier(0);
        fx = fxn;
        if constexpr (REM) yr = yrn;
#pragma unroll
        for (int i = 0; i < NA; ++i) ya[i] = yan[i];
        if constexpr (!DIAG) {
#pragma unroll
            for (int j = 0; j < NB; ++j) yb[j] = ybn[j];
        }
    }
    // REM: add the four voxel groups of the wave (lanes 16 apart); partners add
    // the same two values, so every group ends with the same bits
    constexpr int NQ = REM ? (NA + 4) / 4 : 0;   // f4 slots of the NA + 1 sums
    f4 cq[NQ > 0 ? NQ : 1];
    if constexpr (REM) {
#pragma unroll
        for (int i = 0; i <= NA; ++i) {
            float v = cacc[i];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            cacc[i] = v;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) cq[q][e] = 4 * q + e <= NA ? cacc[4 * q + e] : 0.f;
    }
    constexpr int NT = DIAG ? NA * (NA + 1) / 2 : NA * NB;   // product tiles

    // the waves' accumulators are added in LDS in wave order; then every wave
    // writes a quarter of the tiles
#pragma unroll 1
    for (int wv = 0; wv < 4; ++wv) {
        if (wave == wv) {
            int t = 0;
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int j = DIAG ? i : 0; j < NB; ++j, ++t) {
                    f4 v = acc[i][j];
                    if (wv > 0) v += red[t * 64 + lane];
                    red[t * 64 + lane] = v;
                }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                f4 v = cq[q];
                if (wv > 0) v += red[(NT + q) * 64 + lane];
                red[(NT + q) * 64 + lane] = v;
            }
        }
        __syncthreads();
    }
    int t = 0;
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = DIAG ? i : 0; j < NB; ++j, ++t) {
            if ((t & 3) != wave) continue;
            const f4 v = red[t * 64 + lane];
            const int ib = 16 * (tb0 + j) + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ia = 16 * (ta0 + i) + 4 * (lane >> 4) + r;
                if (ia <= ib && ib < g.M) out[tri_row(ia, g.M) + (ib - ia)] = v[r];
            }
        }
    // REM: (row a, M - 1) for the band's rows from lanes 0..15; the corner from the last band
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (((NT + q) & 3) != wave || lane >= 16) continue;
        const f4 v = red[(NT + q) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * q + e;
            if (k < NA) {
                const int ia = 16 * (ta0 + k) + lane;
                out[tri_row(ia, g.M) + (g.M - 1 - ia)] = v[e];
            } else if (k == NA && lane == 0 && ta0 + NA == a.n16) {
                out[tri_row(g.M - 1, g.M)] = v[e];
            }
        }
    }
}

// Forward: block = (box, super-tile) x channel x field, four waves.  DIAG: the
// super-tiles on the diagonal (row band = column band); else those above it,
// whose row band is always whole.  The valid column tiles of the band select a
// fully unrolled body.
template <bool SOFT, bool DIAG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DIAG ? 2 : 1))) void k_s3_fwd_mf(S3MfArgs a)
{
    extern __shared__ float4 sm4[];
    const S3Geo &g = a.g;
    const int nsup = DIAG ? a.nst : a.nst * (a.nst - 1) / 2;
    const int64_t chunk = blockIdx.x / nsup;
    int sup = (int)(blockIdx.x % nsup);
    int ba = sup, bb = sup;
    if constexpr (!DIAG) {   // off-diagonal super-tile (ba, bb), ba < bb, ba-major
        ba = 0;
        while (sup >= a.nst - 1 - ba) {
            sup -= a.nst - 1 - ba;
            ++ba;
        }
        bb = ba + 1 + sup;
    }
    const int ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    const int tv = a.ed[0] * a.ed[1] * a.ed[2];
    float *T = reinterpret_cast<float *>(sm4);
    f4 *red = reinterpret_cast<f4 *>(sm4 + (tv + 4) / 4);
    mf_load_tile(a, a.phi + (b * a.C + ch) * g.N, chunk, T);
    __syncthreads();
    const int ta0 = ba * kSup, tb0 = bb * kSup;
    float *out = a.part + ((b * a.C + ch) * a.chunks + chunk) * g.K3;
    const bool rem = DIAG && a.rem;
    switch (min(kSup, a.n16 - tb0)) {
#define DMCR_FWD_CASE(n)                                                               \
    case n:                                                                            \
        if constexpr (DIAG) {                                                          \
            if (rem) {                                                                 \
                fwd_super<SOFT, true, n, n, true>(a, T, red, ta0, tb0, out);           \
                break;                                                                 \
            }                                                                          \
        }                                                                              \
        fwd_super<SOFT, DIAG, DIAG ? n : kSup, n>(a, T, red, ta0, tb0, out);           \
        break;
        DMCR_FWD_CASE(1)
        DMCR_FWD_CASE(2)
        DMCR_FWD_CASE(3)
        DMCR_FWD_CASE(4)
        DMCR_FWD_CASE(5)
        DMCR_FWD_CASE(6)
#undef DMCR_FWD_CASE
    }
}

// One pass of the adjoint over NC vector tiles from column 16 c0t: D = E Gf / N
// for the wave's 64 voxels (four 16-voxel row tiles, K = 4 vectors d per
// instruction), then Q stored and the local term added into loc.  A step reads
// the next step's raw tile values and cotangent rows (and the displacement
// offsets of the step after) before running the current products.
//
// REM (the last pass when M = 16 n16 + 1): each lane also sums E[x][d] Gf[d][M-1]
// for its A voxels by FMAs on the A operands it holds; dcol[i] returns N D[x][M-1]
// for x = voxel 16 i + (lane & 15) of the group, the same in all four lane groups.
template <bool SOFT, bool GL, int NC, bool REM = false>
__device__ __forceinline__ void adj_pass(const S3MfArgs &a, const float *T, const int *offs, const float *Gf,
                                         const float *Gs, float *Q, int c0t, const int (&baseA)[4],
                                         const int (&baseO)[4], const int64_t (&gO)[4], float (&loc)[4][4],
                                         float (&dcol)[4])
{
    const S3Geo &g = a.g;
    const int lane = threadIdx.x & 63;
    const int col = 16 * c0t + (lane & 15);
    const int zero = a.ed[0] * a.ed[1] * a.ed[2];
    f4 acc[4][NC];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    float dacc[4] = {0.f, 0.f, 0.f, 0.f};
    float fx[4];   // phi at the four A voxels (the soft threshold's first point)
    if constexpr (SOFT) {
#pragma unroll
        for (int i = 0; i < 4; ++i) fx[i] = T[baseA[i]];
    }
    const int steps = a.Kp / 4;
    auto fetch = [&](int s, int od, float (&ya_)[4], float (&bv_)[NC], float &br_) {
        const int d = 4 * s + (lane >> 4);
        const bool ok = d < g.M;
#pragma unroll
        for (int j = 0; j < NC; ++j) bv_[j] = GL ? Gs[d * a.gs + col + 16 * j] : Gf[(int64_t)d * a.Mp + col + 16 * j];
        if constexpr (REM) br_ = GL ? Gs[d * a.gs + g.M - 1] : Gf[(int64_t)d * a.Mp + g.M - 1];
#pragma unroll
        for (int i = 0; i < 4; ++i) ya_[i] = T[ok ? baseA[i] + od : zero];
    };
    float ya[4], bv[NC], br = 0.f;
    int odn = offs[4 * min(1, steps - 1) + (lane >> 4)];
    fetch(0, offs[lane >> 4], ya, bv, br);
    for (int s = 0; s < steps; ++s) {
        // the last step reads its own operands again: no branch around the reads
        float yan[4], bn[NC], brn = 0.f;
        const int od = odn;
        odn = offs[4 * min(s + 2, steps - 1) + (lane >> 4)];
        fetch(min(s + 1, steps - 1), od, yan, bn, brn);
        __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the products
        float av[4];
        const float m = 4 * s + (lane >> 4) < g.M ? 1.f : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = mf_real<SOFT>(SOFT ? fx[i] : 0.f, ya[i], m, a.sc);
#pragma unroll
        for (int j = 0; j < NC; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
        if constexpr (REM) {
#pragma unroll
            for (int i = 0; i < 4; ++i) dacc[i] = fmaf(av[i], br, dacc[i]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 4; ++i) ya[i] = yan[i];
#pragma unroll
        for (int j = 0; j < NC; ++j) bv[j] = bn[j];
        if constexpr (REM) br = brn;
    }
    if constexpr (REM) {   // the four lane groups hold d = 4 s + group: add them
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float v = dacc[i];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            dcol[i] = v;
        }
    }
    // D[x][c] = acc / N for x = 16 i + 4 (lane >> 4) + r of the group, c = col + 16 j
    const float hq = 0.5f * a.sc.c1 * a.sc.alpha;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        const int c = col + 16 * j;
        if (c >= g.M) continue;
        const int oc = offs[c];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f4 q;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int base = baseO[i] + r;   // four voxels along the innermost axis
                const float D = acc[i][j][r] * a.invN;
                if constexpr (SOFT) {
                    const float sg = soft_sig(T[base] + T[base + oc], a.sc);
                    q[r] = hq * sg * (1.f - sg) * D;
                    loc[i][r] += q[r];
                } else {
                    q[r] = T[base] * D;
                    loc[i][r] += 0.5f * T[base + oc] * D;
                }
            }
            *reinterpret_cast<f4 *>(Q + (int64_t)c * g.N + gO[i]) = q;
        }
    }
}

// Adjoint: block = box x channel x field, nw waves; a wave takes 64 voxels of
// the box at a time and the vectors in passes of up to kSup 16-wide tiles.  GL:
// the block builds the expanded cotangent in LDS (rows a.gs apart) from the
// packed one; else it reads the expanded copy in the workspace.
template <bool SOFT, bool GL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_s3_adj_mf(S3MfArgs a)
{
    extern __shared__ float4 sm4[];
    const S3Geo &g = a.g;
    const int64_t chunk = blockIdx.x;
    const int ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    const int tv = a.ed[0] * a.ed[1] * a.ed[2];
    float *T = reinterpret_cast<float *>(sm4);
    int *offs = reinterpret_cast<int *>(T + tv + 1);   // [Kp] tile offset of r_d (0 past M)
    const int64_t bc = b * a.C + ch;
    float *Gs = reinterpret_cast<float *>(offs + a.Kp);   // GL: [Kp][gs]
    mf_load_tile(a, a.phi + bc * g.N, chunk, T);
    for (int d = threadIdx.x; d < a.Kp; d += blockDim.x) offs[d] = d < g.M ? mf_off(a, d) : 0;
    const float *Gf = a.Gf + bc * (int64_t)a.Kp * a.Mp;
    if constexpr (GL) {   // Gs[d][c] = G(min, max), doubled on the diagonal, zero in the padding;
        // sixteen entries per thread and batch, their reads issued before the stores
        constexpr int U = 16;
        const int64_t gp = b * a.Kstride + a.off + ch * g.K3;
        const int tot = a.Kp * a.Mp;
        for (int base = threadIdx.x; base < tot; base += U * blockDim.x) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = base + u * blockDim.x;
                const int d = fdivu(idx, a.fd_mp), c = idx - d * a.Mp;
                v[u] = 0.f;
                if (idx < tot && c < g.M && d < g.M) {
                    const int lo = c < d ? c : d, hi = c < d ? d : c;
                    v[u] = s3_cot(a.G, a.St, a.w2, a.invZ, gp + tri_row(lo, g.M) + (hi - lo)) * (c == d ? 2.f : 1.f);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = base + u * blockDim.x;
                const int d = fdivu(idx, a.fd_mp), c = idx - d * a.Mp;
                if (idx < tot) Gs[d * a.gs + c] = v[u];
            }
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    float *Q = a.Q + bc * (int64_t)g.M * g.N;
    for (int grp = wave; grp < a.VB / 64; grp += nw) {
        const int v0 = grp * 64;
        int baseA[4], baseO[4];   // A rows: voxel v0 + 16 i + (lane & 15); outputs from v0 + 16 i + 4 (lane >> 4)
        int64_t gO[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            baseA[i] = mf_base(a, v0 + 16 * i + (lane & 15));
            baseO[i] = mf_base(a, v0 + 16 * i + 4 * (lane >> 4));
            gO[i] = mf_voxel(a, chunk, v0 + 16 * i + 4 * (lane >> 4));
        }
        float loc[4][4], dcol[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) loc[i][r] = 0.f;
        for (int cg = 0; cg * kSup < a.n16; ++cg) {
            const int c0t = cg * kSup;
            const bool rem = a.rem && (cg + 1) * kSup >= a.n16;   // the last pass takes column M - 1
            switch (min(kSup, a.n16 - c0t)) {
#define DMCR_ADJ_CASE(n)                                                                    \
    case n:                                                                                 \
        if (rem)                                                                            \
            adj_pass<SOFT, GL, n, true>(a, T, offs, Gf, Gs, Q, c0t, baseA, baseO, gO, loc, dcol); \
        else                                                                                \
            adj_pass<SOFT, GL, n>(a, T, offs, Gf, Gs, Q, c0t, baseA, baseO, gO, loc, dcol); \
        break;
                DMCR_ADJ_CASE(1)
                DMCR_ADJ_CASE(2)
                DMCR_ADJ_CASE(3)
                DMCR_ADJ_CASE(4)
                DMCR_ADJ_CASE(5)
                DMCR_ADJ_CASE(6)
#undef DMCR_ADJ_CASE
            }
        }
        // sum the local terms over the 16 lanes (columns) of each row group; lane
        // (lane & 15) = 4 i + r then adds voxel (i, r) of its row group
        float mine = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float s = loc[i][r];
                s += __shfl_xor(s, 1);
                s += __shfl_xor(s, 2);
                s += __shfl_xor(s, 4);
                s += __shfl_xor(s, 8);
                if ((lane & 15) == 4 * i + r) mine = s;
            }
        const int vm = v0 + 16 * ((lane & 15) >> 2) + 4 * (lane >> 4) + (lane & 3);
        const int64_t gm = mf_voxel(a, chunk, vm);
        if (a.rem) {
            // column M - 1 of this lane's voxel vm = v0 + 16 im + pm, held by lane pm
            const int im = (lane & 15) >> 2, pm = 4 * (lane >> 4) + (lane & 3);
            float dn = 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = __shfl(dcol[i], pm);
                if (i == im) dn = v;
            }
            const float D = dn * a.invN;
            const int bm = mf_base(a, vm), om = offs[g.M - 1];
            float q;
            if constexpr (SOFT) {
                const float sg = soft_sig(T[bm] + T[bm + om], a.sc);
                q = 0.5f * a.sc.c1 * a.sc.alpha * sg * (1.f - sg) * D;
                mine += q;
            } else {
                q = T[bm] * D;
                mine += 0.5f * T[bm + om] * D;
            }
            Q[(int64_t)(g.M - 1) * g.N + gm] = q;
        }
        a.grad[bc * g.N + gm] += mine;
    }
}

// grad(y) += sum_c Q_c(y - r_c) (the matrix-core adjoint added the local term):
// kShG x 64 voxels per block (fewer when the field is smaller), wave q summing
// c = q, q + 4, ... for each of its voxels; the four sums of a voxel are added in
// wave order
constexpr int kShG = 4;

// voxel groups per block: four on fields of 2^16 voxels and more, fewer below
// (N is a power of two >= 64), so that small fields still spread over the chip
__host__ __device__ __forceinline__ int shift_groups(int64_t N)
{
    const int64_t g = N / (64 * 256);
    return g >= kShG ? kShG : (g >= 2 ? 2 : 1);
}

template <int G>
__global__ __launch_bounds__(256) void k_s3_adj_shift(S3MfArgs a)
{
    __shared__ int3 rv[361];
    __shared__ float part[3][G * 64];
    const S3Geo &g = a.g;
    const int ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    for (int c = threadIdx.x; c < g.M; c += 256) {
        int c0, c1, c2;
        vec_of(g, c, c0, c1, c2);
        rv[c] = int3{c0, c1, c2};
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t bc = b * a.C + ch;
    const float *Qb = a.Q + bc * g.M * g.N;
    int i0[G], i1[G], i2[G];
    float acc[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const int64_t y = ((int64_t)blockIdx.x * G + q) * 64 + lane;
        i2[q] = (int)(y % g.n2);
        i1[q] = (int)((y / g.n2) % g.n1);
        i0[q] = (int)(y / ((int64_t)g.n1 * g.n2));
        acc[q] = 0.f;
    }
#pragma unroll 4
    for (int c = wave; c < g.M; c += 4) {
        const int3 r = rv[c];
        const float *Qc = Qb + (int64_t)c * g.N;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int64_t x = ((int64_t)((i0[q] - r.x) & (g.n0 - 1)) * g.n1 + ((i1[q] - r.y) & (g.n1 - 1))) * g.n2 +
                              ((i2[q] - r.z) & (g.n2 - 1));
            acc[q] += Qc[x];
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int q = 0; q < G; ++q) part[wave - 1][q * 64 + lane] = acc[q];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int64_t y = ((int64_t)blockIdx.x * G + q) * 64 + lane;
            a.grad[bc * g.N + y] += ((acc[q] + part[0][q * 64 + lane]) + part[1][q * 64 + lane]) + part[2][q * 64 + lane];
        }
    }
}

S3Geo make_s3geo(const Plan &p, int l)
{
    const LevelPlan &L = p.lv[l];
    S3Geo g{};
    g.ndim = p.ndim;
    g.n0 = L.n[0];
    g.n1 = L.n[1];
    g.n2 = p.ndim == 3 ? L.n[2] : 1;
    g.N = L.N;
    g.P3 = L.s3P;
    g.box = 2 * L.s3P + 1;
    g.M = L.s3M;
    g.K3 = L.s3K;
    return g;
}

SoftC make_softc(const Plan &p)
{
    const double log2e = 1.4426950408889634074;
    return SoftC{(float)p.alpha, (float)p.c1, (float)p.c2, (float)p.c3, (float)(-0.5 * p.alpha * log2e),
                 (float)(-p.alpha * p.c2 * log2e)};
}

S3MapArgs map_args(const Plan &p, float *S)
{
    S3MapArgs a{};
    a.S = S;
    a.ndim = p.ndim;
    a.C = p.C;
    a.Kstride = p.K;
    a.h = p.fh;
    for (int l = 0; l < p.L; ++l) {
        const LevelPlan &L = p.lv[l];
        a.P3[l] = L.s3P;
        a.M[l] = L.s3M;
        a.P[l] = L.P;
        a.K3[l] = L.s3K;
        a.off3[l] = L.s3off;
        for (int q = 0; q < p.npairs; ++q)
            if (p.pi[q] == p.pj[q]) {
                a.off2[l][p.pi[q]] = L.off[q];
                a.cnt2[l] = L.cnt[q];
            }
    }
    return a;
}

}  // namespace

// Mp = M rounded up to a multiple of 4 (the register tiles)
int s3_Mp(int M) { return (M + 3) / 4 * 4; }

namespace {

int ilog2(int v)
{
    int k = 0;
    while ((1 << (k + 1)) <= v) ++k;
    return k;
}

// box of VB voxels: powers of two dealt out one bit at a time from the innermost
// axis outwards, never beyond an axis' length; false if VB does not fit the level
bool s3_box(const Plan &p, int l, int VB, int bd[3])
{
    const LevelPlan &L = p.lv[l];
    const int n[3] = {L.n[0], L.n[1], p.ndim == 3 ? L.n[2] : 1};
    bd[0] = bd[1] = bd[2] = 1;
    int rem = ilog2(VB);
    const int order3[3] = {2, 1, 0}, order2[2] = {1, 0};
    const int *order = p.ndim == 3 ? order3 : order2;
    while (rem > 0) {
        bool grew = false;
        for (int t = 0; t < p.ndim && rem > 0; ++t) {
            const int ax = order[t];
            if (2 * bd[ax] <= n[ax]) {
                bd[ax] *= 2;
                --rem;
                grew = true;
            }
        }
        if (!grew) return false;
    }
    return true;
}

int tile_floats(const Plan &p, int l, const int bd[3])
{
    const int P3 = p.lv[l].s3P;
    int v = 1;
    for (int ax = 0; ax < 3; ++ax) v *= bd[ax] + ((ax < p.ndim && (p.ndim == 3 || ax < 2)) ? 2 * P3 : 0);
    return v;
}

// LDS of the matrix-core kernels: the field tile and its zero cell, then the
// wave sums (forward) or the displacement offsets (adjoint)
size_t fwd_mf_lds(int tv, bool diag)
{
    // a diagonal super-tile also carries the remainder sums: two more slots
    return (size_t)(tv + 4) / 4 * 16 + (size_t)(diag ? kSup * (kSup + 1) / 2 + 2 : kSup * kSup) * 64 * 16;
}
size_t adj_mf_lds(int tv, int Kp) { return (size_t)(tv + 1) * 4 + (size_t)Kp * 4; }
// row stride of the cotangent's LDS copy, and whether the copy is made
int adj_gs(int Mp) { return Mp + (((16 - Mp) % 32) + 32) % 32; }
bool adj_gl(int tv, int Kp, int Mp)
{
    return Mp <= 128 && adj_mf_lds(tv, Kp) + (size_t)Kp * adj_gs(Mp) * 4 <= 48 * 1024;
}

}  // namespace

// Matrix cores when every voxel box is whole (N >= 64) and the innermost axis
// holds the adjoint's four-voxel stores (length >= 4); the box takes N / 64
// voxels, clamped to [64, 1024], for the forward and the adjoint alike, so a
// field's blocks and sums do not depend on the batch.
bool s3_configure(Plan &p, int l)
{
    LevelPlan &L = p.lv[l];
    const int M = L.s3M;
    if (M > 361) return false;   // 2-D P3 <= 9, 3-D P3 <= 3
    const int inner = L.n[p.ndim - 1];
    L.s3mf = 0;
    if (L.N >= 64 && inner >= 4) {
        int VB = 64;
        while (VB < 1024 && (int64_t)VB * 2 <= L.N / 64) VB *= 2;
        int bd[3];
        const int n16 = (M + 15) / 16;
        const int Kp = (M + 3) / 4 * 4;
        if (s3_box(p, l, VB, bd) && bd[p.ndim == 3 ? 2 : 1] >= 4) {
            const int tv = tile_floats(p, l, bd);
            if (fwd_mf_lds(tv, false) <= (size_t)kMfLds && adj_mf_lds(tv, Kp) <= (size_t)kMfLds) {
                L.s3mf = 1;
                L.s3VB = L.s3VBa = VB;
                for (int ax = 0; ax < 3; ++ax) L.s3bf[ax] = L.s3ba[ax] = bd[ax];
                L.s3Kp = Kp;
                L.s3Mp = 16 * n16;
                L.s3chunks = L.N / VB;
                return true;
            }
        }
    }
    const int64_t Mp = s3_Mp(M);
    int vb = 128, vba = 64;
    while (vb > 4 && ((size_t)(vb * Mp + vb) * sizeof(float) > kS3Lds || vb > L.N)) vb /= 2;
    while (vba > 4 && ((size_t)(vba * M) * sizeof(float) > kS3Lds || vba > L.N)) vba /= 2;
    if ((size_t)(vb * Mp + vb) * sizeof(float) > kS3Lds || (size_t)(vba * M) * sizeof(float) > kS3Lds) return false;
    if (vb < 4 || vba < 4 || L.N % vb || L.N % vba) return false;   // whole 4-voxel tiles
    L.s3VB = vb;
    L.s3VBa = vba;
    L.s3Kp = M;
    L.s3Mp = (int)Mp;
    L.s3chunks = L.N / vb;
    return true;
}

namespace {

S3MfArgs mf_args(const Plan &p, int l, const int bd[3])
{
    const LevelPlan &L = p.lv[l];
    S3MfArgs a{};
    a.g = make_s3geo(p, l);
    a.sc = make_softc(p);
    a.C = p.C;
    const int n[3] = {a.g.n0, a.g.n1, a.g.n2};
    a.VB = 1;
    for (int ax = 0; ax < 3; ++ax) {
        a.bd[ax] = bd[ax];
        a.lb[ax] = ilog2(bd[ax]);
        a.nb[ax] = n[ax] / bd[ax];
        a.hl[ax] = (p.ndim == 3 || ax < 2) ? L.s3P : 0;
        a.ed[ax] = bd[ax] + 2 * a.hl[ax];
        a.VB *= bd[ax];
    }
    a.chunks = L.N / a.VB;
    a.rem = (L.s3M > 16 && L.s3M % 16 == 1) ? 1 : 0;
    a.n16 = a.rem ? L.s3M / 16 : (L.s3M + 15) / 16;
    a.nst = (a.n16 + kSup - 1) / kSup;
    a.Kp = L.s3Kp;
    a.Mp = L.s3Mp;
    a.invN = (float)(1.0 / (double)L.N);
    a.fd_rl = make_fastdivu(p.ndim == 3 ? a.ed[2] : a.ed[1]);
    a.fd_e1 = make_fastdivu(a.ed[1]);
    a.fd_mp = make_fastdivu(a.Mp);
    return a;
}

hipError_t s3_reduce_level(const Plan &p, int l, const float *part, float *S, hipStream_t st)
{
    const LevelPlan &L = p.lv[l];
    S3RedArgs r{};
    r.part = part;
    r.S = S;
    r.C = p.C;
    r.chunks = L.s3chunks;
    r.K3 = L.s3K;
    r.Kstride = p.K;
    r.off = L.s3off;
    r.invN = 1.0 / (double)L.N;
    const dim3 rg((unsigned)((L.s3K + kRK - 1) / kRK), (unsigned)p.C, (unsigned)p.B);
    return launch("s3_reduce", (double)p.B * p.C * L.s3chunks * L.s3K * 4, k_s3_reduce, rg, dim3(kT3), 0, st, r);
}

hipError_t s3_forward_mf(const Plan &p, int l, const float *phi, float *S, const Ws &ws, hipStream_t st)
{
    const LevelPlan &L = p.lv[l];
    S3MfArgs a = mf_args(p, l, L.s3bf);
    a.phi = phi;
    a.part = ws.at<float>(L.s3part);
    const bool soft = p.desc != DMCR_DESC_S2;
    const int tv = a.ed[0] * a.ed[1] * a.ed[2];
    const double bytes = (double)p.B * p.C * (L.N * 4 + a.chunks * L.s3K * 4);
    const dim3 gd((unsigned)(a.chunks * a.nst), (unsigned)p.C, (unsigned)p.B);
    hipError_t e = soft ? launch("s3_fwd_mf_soft", bytes, k_s3_fwd_mf<true, true>, gd, dim3(256), fwd_mf_lds(tv, true),
                                 st, a)
                        : launch("s3_fwd_mf", bytes, k_s3_fwd_mf<false, true>, gd, dim3(256), fwd_mf_lds(tv, true),
                                 st, a);
    if (e != hipSuccess) return e;
    if (a.nst > 1) {
        const dim3 go((unsigned)(a.chunks * (a.nst * (a.nst - 1) / 2)), (unsigned)p.C, (unsigned)p.B);
        e = soft ? launch("s3_fwd_mf_soft_off", 0.0, k_s3_fwd_mf<true, false>, go, dim3(256), fwd_mf_lds(tv, false), st,
                          a)
                 : launch("s3_fwd_mf_off", 0.0, k_s3_fwd_mf<false, false>, go, dim3(256), fwd_mf_lds(tv, false), st, a);
        if (e != hipSuccess) return e;
    }
    return s3_reduce_level(p, l, a.part, S, st);
}

hipError_t launch_shift(const Plan &p, int l, const S3MfArgs &a, hipStream_t st)
{
    const LevelPlan &L = p.lv[l];
    const int G = shift_groups(L.N);
    const dim3 gg((unsigned)(L.N / 64 / G), (unsigned)p.C, (unsigned)p.B);
    const double bytes = (double)p.B * p.C * (L.s3M * (double)L.N * 4 + L.N * 8.0);
    if (G == 4) return launch("s3_adj_shift", bytes, k_s3_adj_shift<4>, gg, dim3(256), 0, st, a);
    if (G == 2) return launch("s3_adj_shift", bytes, k_s3_adj_shift<2>, gg, dim3(256), 0, st, a);
    return launch("s3_adj_shift", bytes, k_s3_adj_shift<1>, gg, dim3(256), 0, st, a);
}

hipError_t s3_adjoint_mf(const Plan &p, int l, const float *phi, const float *G, float *grad, const Ws &ws,
                         hipStream_t st, const double *St)
{
    const LevelPlan &L = p.lv[l];
    S3MfArgs a = mf_args(p, l, L.s3ba);
    a.phi = phi;
    a.Gf = ws.at<float>(L.s3G);
    a.G = G;
    a.St = St;
    a.w2 = p.w[l] * p.w[l];
    a.invZ = 1.0 / p.Z;
    a.Kstride = p.K;
    a.off = L.s3off;
    a.Q = ws.at<float>(L.s3Q);
    a.grad = grad;
    const bool soft = p.desc != DMCR_DESC_S2;
    const int tv = a.ed[0] * a.ed[1] * a.ed[2];
    const int nw = std::min(4, a.VB / 64);
    const dim3 grid((unsigned)a.chunks, (unsigned)p.C, (unsigned)p.B);
    const double qbytes = (double)p.B * p.C * (L.s3M * (double)L.N * 4 + L.N * 12.0);
    a.gs = adj_gs(a.Mp);
    hipError_t e;
    if (nw == 4 && adj_gl(tv, a.Kp, a.Mp)) {   // four waves share the expanded cotangent built in LDS
        const size_t lds = adj_mf_lds(tv, a.Kp) + (size_t)a.Kp * a.gs * 4;
        e = soft ? launch("s3_adj_mf_soft", qbytes, k_s3_adj_mf<true, true>, grid, dim3(64 * nw), lds, st, a)
                 : launch("s3_adj_mf", qbytes, k_s3_adj_mf<false, true>, grid, dim3(64 * nw), lds, st, a);
        if (e != hipSuccess) return e;
        return launch_shift(p, l, a, st);
    }
    // the expanded cotangent in the workspace, as for the FMA kernels but with Kp rows and Mp columns
    S3AdjArgs x{};
    x.g = a.g;
    x.G = G;
    x.St = St;
    x.w2 = a.w2;
    x.invZ = a.invZ;
    x.Gf = ws.at<float>(L.s3G);
    x.C = p.C;
    x.Mp = L.s3Mp;
    x.Kp = L.s3Kp;
    x.Kstride = p.K;
    x.off = L.s3off;
    const int64_t gfn = (int64_t)L.s3Kp * L.s3Mp;
    const dim3 eg((unsigned)std::min<int64_t>(64, (gfn + kT3 - 1) / kT3), (unsigned)p.C, (unsigned)p.B);
    e = launch("s3_expand", (double)p.B * p.C * (L.s3K + (double)gfn) * 4, k_s3_expand, eg, dim3(kT3), 0, st, x);
    if (e != hipSuccess) return e;
    const size_t lds = adj_mf_lds(tv, a.Kp);
    e = soft ? launch("s3_adj_mf_soft", qbytes, k_s3_adj_mf<true, false>, grid, dim3(64 * nw), lds, st, a)
             : launch("s3_adj_mf", qbytes, k_s3_adj_mf<false, false>, grid, dim3(64 * nw), lds, st, a);
    if (e != hipSuccess) return e;
    return launch_shift(p, l, a, st);
}

}  // namespace

hipError_t s3_forward_level(const Plan &p, int l, const float *phi, float *S, const Ws &ws, hipStream_t st)
{
    const LevelPlan &L = p.lv[l];
    if (L.s3mf) return s3_forward_mf(p, l, phi, S, ws, st);
    S3FwdArgs a{};
    a.g = make_s3geo(p, l);
    a.sc = make_softc(p);
    a.phi = phi;
    a.part = ws.at<float>(L.s3part);
    a.C = p.C;
    a.VB = L.s3VB;
    a.Mp = s3_Mp(L.s3M);
    a.chunks = L.s3chunks;
    const size_t lds = (size_t)(a.VB * a.Mp + a.VB) * sizeof(float);
    const dim3 grid((unsigned)a.chunks, (unsigned)p.C, (unsigned)p.B);
    const double bytes = (double)p.B * p.C * (L.N * 4 + a.chunks * L.s3K * 4);
    hipError_t e = (p.desc == DMCR_DESC_S2)
                       ? launch("s3_fwd", bytes, k_s3_fwd<false>, grid, dim3(kT3), lds, st, a)
                       : launch("s3_fwd_soft", bytes, k_s3_fwd<true>, grid, dim3(kT3), lds, st, a);
    if (e != hipSuccess) return e;
    return s3_reduce_level(p, l, a.part, S, st);
}

hipError_t s3_adjoint_level(const Plan &p, int l, const float *phi, const float *G, float *grad, const Ws &ws,
                            hipStream_t st, const double *St)
{
    const LevelPlan &L = p.lv[l];
    if (L.s3mf) return s3_adjoint_mf(p, l, phi, G, grad, ws, st, St);
    S3AdjArgs a{};
    a.g = make_s3geo(p, l);
    a.sc = make_softc(p);
    a.phi = phi;
    a.G = G;
    a.St = St;
    a.w2 = p.w[l] * p.w[l];
    a.invZ = 1.0 / p.Z;
    a.Gf = ws.at<float>(L.s3G);
    a.Q = ws.at<float>(L.s3Q);
    a.R = (p.desc == DMCR_DESC_S2) ? ws.at<float>(L.s3R) : nullptr;
    a.grad = grad;
    a.C = p.C;
    a.VB = L.s3VBa;
    a.Mp = s3_Mp(L.s3M);
    a.Kp = L.s3M;
    a.Kstride = p.K;
    a.off = L.s3off;
    a.invN = (float)(1.0 / (double)L.N);
    const dim3 eg((unsigned)std::min<int64_t>(64, ((int64_t)L.s3M * a.Mp + kT3 - 1) / kT3), (unsigned)p.C,
                  (unsigned)p.B);
    hipError_t e = launch("s3_expand", (double)p.B * p.C * (L.s3K + (double)L.s3M * a.Mp) * 4, k_s3_expand, eg,
                          dim3(kT3), 0, st, a);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)(a.VB * a.g.M) * sizeof(float);
    const dim3 grid((unsigned)(L.N / a.VB), (unsigned)p.C, (unsigned)p.B);
    const double qbytes = (double)p.B * p.C * L.s3M * L.N * 4 * (p.desc == DMCR_DESC_S2 ? 2 : 1);
    const bool soft = p.desc != DMCR_DESC_S2;
    e = soft ? launch("s3_adj_terms_soft", qbytes, k_s3_adj_terms<true>, grid, dim3(kT3), lds, st, a)
             : launch("s3_adj_terms", qbytes, k_s3_adj_terms<false>, grid, dim3(kT3), lds, st, a);
    if (e != hipSuccess) return e;
    const dim3 gg((unsigned)((L.N + kT3 - 1) / kT3), (unsigned)p.C, (unsigned)p.B);
    const double gbytes = qbytes + (double)p.B * p.C * L.N * 8;
    return soft ? launch("s3_adj_gather_soft", gbytes, k_s3_adj_gather<true>, gg, dim3(kT3), 0, st, a)
                : launch("s3_adj_gather", gbytes, k_s3_adj_gather<false>, gg, dim3(kT3), 0, st, a);
}

hipError_t launch_s3_map(const Plan &p, float *S, hipStream_t st)
{
    const S3MapArgs a = map_args(p, S);
    return launch("s3_map", (double)p.B * p.K * 8, k_s3_map, dim3((unsigned)p.L, (unsigned)p.C, (unsigned)p.B),
                  dim3(kT3), 0, st, a);
}

hipError_t launch_s3_map_adjoint(const Plan &p, float *G, hipStream_t st)
{
    const S3MapArgs a = map_args(p, G);
    const dim3 grid((unsigned)p.L, (unsigned)p.C, (unsigned)p.B);
    hipError_t e = launch("s3_map_adj", (double)p.B * p.K * 8, k_s3_map_adj_gather, grid, dim3(kT3), 0, st, a);
    if (e != hipSuccess) return e;
    return launch("s3_map_adj_scale", (double)p.B * p.K * 8, k_s3_map_adj_scale, grid, dim3(kT3), 0, st, a);
}

}  // namespace dmcr
