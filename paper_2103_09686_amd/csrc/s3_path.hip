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
// Both contractions run register-blocked: each thread owns a 4 x 4 tile of the
// output and reads two float4 per 16 multiply-adds.
#include <algorithm>

#include "dmcr_internal.h"

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

struct SoftC {
    float alpha, c1, c2, c3;
};

__device__ __forceinline__ float soft_sig(float u, const SoftC &s)
{
    return __builtin_amdgcn_rcpf(1.f + __expf(-s.alpha * (u + s.c2)));
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
        return fmaf(sc.c1, soft_sig(0.5f * (f[x] + fy), sc), sc.c3);
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

struct S3AdjArgs {
    S3Geo g;
    SoftC sc;
    const float *phi;
    const float *G;     // cotangent [B][Kstride]
    float *Gf;          // [B][C][M][Mp] full symmetric cotangent, diagonal doubled
    float *Q, *R;       // [B][C][M][N]
    float *grad;        // level gradient [B][C][N] (added to)
    int C, VB, Mp;
    int64_t Kstride, off;
    float invN;
};

// Gf[c][d] = G(min, max), doubled on the diagonal, zero in the padding columns
__global__ __launch_bounds__(kT3) void k_s3_expand(S3AdjArgs a)
{
    const S3Geo &g = a.g;
    const int ch = blockIdx.y;
    const int64_t b = blockIdx.z;
    const float *Gb = a.G + b * a.Kstride + a.off + ch * g.K3;
    float *out = a.Gf + (b * a.C + ch) * (int64_t)g.M * a.Mp;
    for (int64_t idx = (int64_t)blockIdx.x * kT3 + threadIdx.x; idx < (int64_t)g.M * a.Mp;
         idx += (int64_t)gridDim.x * kT3) {
        const int c = (int)(idx / a.Mp), d = (int)(idx % a.Mp);
        float v = 0.f;
        if (d < g.M) {
            const int lo = c < d ? c : d, hi = c < d ? d : c;
            v = Gb[tri_row(lo, g.M) + (hi - lo)] * (c == d ? 2.f : 1.f);
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
                    const float sg = soft_sig(0.5f * (f[x] + f[shift(g, x, c0, c1, c2)]), a.sc);
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

SoftC make_softc(const Plan &p) { return SoftC{(float)p.alpha, (float)p.c1, (float)p.c2, (float)p.c3}; }

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

bool s3_supported(const Plan &p, int l, int *VB, int *VBa)
{
    const LevelPlan &L = p.lv[l];
    const int64_t M = L.s3M, Mp = s3_Mp(L.s3M);
    if (M > 361) return false;   // 2-D P3 <= 9, 3-D P3 <= 3
    int vb = 128, vba = 64;
    while (vb > 4 && ((size_t)(vb * Mp + vb) * sizeof(float) > kS3Lds || vb > L.N)) vb /= 2;
    while (vba > 4 && ((size_t)(vba * M) * sizeof(float) > kS3Lds || vba > L.N)) vba /= 2;
    if ((size_t)(vb * Mp + vb) * sizeof(float) > kS3Lds || (size_t)(vba * M) * sizeof(float) > kS3Lds) return false;
    if (vb < 4 || vba < 4 || L.N % vb || L.N % vba) return false;   // whole 4-voxel tiles
    *VB = vb;
    *VBa = vba;
    return true;
}

hipError_t s3_forward_level(const Plan &p, int l, const float *phi, float *S, const Ws &ws, hipStream_t st)
{
    const LevelPlan &L = p.lv[l];
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
    S3RedArgs r{};
    r.part = a.part;
    r.S = S;
    r.C = p.C;
    r.chunks = a.chunks;
    r.K3 = L.s3K;
    r.Kstride = p.K;
    r.off = L.s3off;
    r.invN = 1.0 / (double)L.N;
    const dim3 rg((unsigned)((L.s3K + kRK - 1) / kRK), (unsigned)p.C, (unsigned)p.B);
    return launch("s3_reduce", (double)p.B * p.C * a.chunks * L.s3K * 4, k_s3_reduce, rg, dim3(kT3), 0, st, r);
}

hipError_t s3_adjoint_level(const Plan &p, int l, const float *phi, const float *G, float *grad, const Ws &ws,
                            hipStream_t st)
{
    const LevelPlan &L = p.lv[l];
    S3AdjArgs a{};
    a.g = make_s3geo(p, l);
    a.sc = make_softc(p);
    a.phi = phi;
    a.G = G;
    a.Gf = ws.at<float>(L.s3G);
    a.Q = ws.at<float>(L.s3Q);
    a.R = (p.desc == DMCR_DESC_S2) ? ws.at<float>(L.s3R) : nullptr;
    a.grad = grad;
    a.C = p.C;
    a.VB = L.s3VBa;
    a.Mp = s3_Mp(L.s3M);
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
