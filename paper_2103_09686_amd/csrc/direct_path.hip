// Direct (shifted-product) path for short correlation ranges: the paper's own
// convolve-and-reduce of Sec. 3.2.3 (eq. convdef) with the sparse two-point
// masks written as explicit shifts instead of dense mask convolutions.
// The pair term is either the product a b (S2) or, for the soft-threshold
// descriptor of Sec. 3.2.4, f((a + b) / 2)^2 with the logistic f; its
// derivative with respect to either end is b, or f f' at (a + b) / 2.
//
// Forward: one block per (spatial tile, chunk of displacements, batch x pair).
// The tile of phi_i and the tile of phi_j with a halo of P (periodic) sit in
// LDS; each thread owns one displacement r and accumulates
// sum_{x in tile} phi_i(x) phi_j(x + r); phi_i(x) is a broadcast read.  Each
// slab of the tile (first tile axis fixed: 16 terms in 2-D, 64 in 3-D) is
// summed in float32 and the slabs in float64, so that a tile partial carries
// float32 rounding of short sums only; tile partials are summed in float64, in
// tile order, by a second kernel.
// Adjoint: one block per (tile, output channel, batch); each thread owns one
// output voxel and accumulates sum_j sum_r K_cj(r) phi_j(x + r) with the
// cotangent box K_cj read through uniform (scalar) loads.
#include "dmcr_internal.h"

namespace dmcr {

namespace {

constexpr int kT = 256;                 // threads per block
constexpr size_t kDirectLds = 64 * 1024;

struct Geo {
    int ndim;
    int n0, n1, n2;     // level shape (2-D: n2 = 1)
    int t0, t1, t2;     // tile edge
    int h0, h1, h2;     // halo tile edge = t + 2P (2-D: h2 = t2 = 1)
    int p1;             // LDS pitch of the halo's axis-1 index (halo_pitch1), >= h1
    int P, box;
    int nt0, nt1, nt2;  // tiles per axis
};

__device__ __forceinline__ int wrapi(int i, int n)
{
    int m = i % n;
    return m < 0 ? m + n : m;
}

// Load the halo tile of `f` (one channel, [n0][n1][n2]) whose origin is the
// tile origin minus P, into H[h0][p1][h2] (columns h1 .. p1 - 1 unused).
// i = (x d1 + y) d2 + z split into (x, y, z); in 2-D (d2 = 1) with one division
__device__ __forceinline__ void split3(int i, int d1, int d2, bool two_d, int &x, int &y, int &z)
{
    if (two_d) {
        x = i / d1;
        y = i - x * d1;
        z = 0;
    } else {
        z = i % d2;
        const int r = i / d2;
        y = r % d1;
        x = r / d1;
    }
}

template <int NT = kT>
__device__ __forceinline__ void load_halo(const Geo &g, const float *__restrict__ f, int o0, int o1,
                                          int o2, float *H)
{
    if (g.ndim == 2) {
        // halo rows by wave, columns by lane: no index division, and the periodic
        // wrap is one conditional add or subtract (the index lies in [-P, n + P)
        // and P < n / 2)
        const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        for (int x = wave; x < g.h0; x += NT / 64) {
            int i0 = o0 + x - g.P;
            i0 = i0 < 0 ? i0 + g.n0 : (i0 >= g.n0 ? i0 - g.n0 : i0);
            const float *row = f + (int64_t)i0 * g.n1;
            for (int y = lane; y < g.h1; y += 64) {
                int i1 = o1 + y - g.P;
                i1 = i1 < 0 ? i1 + g.n1 : (i1 >= g.n1 ? i1 - g.n1 : i1);
                H[x * g.p1 + y] = row[i1];
            }
        }
        return;
    }
    const int vol = g.h0 * g.h1 * g.h2;
    for (int idx = threadIdx.x; idx < vol; idx += NT) {
        const int z = idx % g.h2;
        const int r = idx / g.h2;
        const int y = r % g.h1;
        const int x = r / g.h1;
        const int i0 = wrapi(o0 + x - g.P, g.n0);
        const int i1 = wrapi(o1 + y - g.P, g.n1);
        const int i2 = (g.ndim == 3) ? wrapi(o2 + z - g.P, g.n2) : 0;
        H[(x * g.p1 + y) * g.h2 + z] = f[((int64_t)i0 * g.n1 + i1) * g.n2 + i2];
    }
}

// logistic soft threshold f(u) = c1 / (1 + exp(-alpha (u + c2))) + c3 of the pair
// mean u = (a + b) / 2, its exponent's constants folded:
//   exp(-alpha ((a + b) / 2 + c2)) = 2^(k1 (a + b) + k0),
//   k1 = -alpha log2(e) / 2,  k0 = -alpha c2 log2(e);
// c1a = c1 alpha, the constant of f'(u) = c1 alpha sigma (1 - sigma)
struct Soft {
    float k1, k0, c1, c3, c1a;
};

// sigma = 1 / (1 + 2^z)
__device__ __forceinline__ float soft_sigma2(float z)
{
    return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(z));
}

struct DirFwdArgs {
    Soft soft;
    Geo g;
    const float *phi;   // level field [B][C][n..]
    double *part;       // [B*npairs][ntiles][kmax]
    int C, npairs;
    int pi[kMaxPairs], pj[kMaxPairs];
    int auto_mask;
    int64_t N, ntiles, kmax, center;
    int64_t cnt[kMaxPairs];
};

// pair term of the forward sum
template <bool SOFT>
__device__ __forceinline__ float pair_term(float a, float b, const Soft &s)
{
    if constexpr (SOFT) {   // f(u)^2
        const float f = fmaf(s.c1, soft_sigma2(fmaf(a + b, s.k1, s.k0)), s.c3);
        return f * f;
    } else {
        return a * b;
    }
}

// TX, TY, TZ: the tile edge when it is the full tile (16 x 16 or 4 x 8 x 8), so the
// tile loops unroll and the LDS reads batch; 0 for grids smaller than one tile.
template <bool SOFT, int TX, int TY, int TZ>
__global__ __launch_bounds__(kT) void k_direct_fwd(DirFwdArgs a)
{
    extern __shared__ float sm[];
    const Geo &g = a.g;
    const int tile = blockIdx.x;
    const int bp = blockIdx.z;
    const int p = bp % a.npairs;
    const int64_t b = bp / a.npairs;
    int tx, ty, tz;
    split3(tile, g.nt1, g.nt2, g.ndim == 2, tx, ty, tz);
    const int o0 = tx * g.t0, o1 = ty * g.t1, o2 = tz * g.t2;
    const int tvol = g.t0 * g.t1 * g.t2;
    float *Ta = sm;
    float *Hb = sm + tvol;
    const float *fa = a.phi + (b * a.C + a.pi[p]) * a.N;
    const float *fb = a.phi + (b * a.C + a.pj[p]) * a.N;
    for (int idx = threadIdx.x; idx < tvol; idx += kT) {
        int x, y, z;
        split3(idx, g.t1, g.t2, g.ndim == 2, x, y, z);
        Ta[idx] = fa[((int64_t)(o0 + x) * g.n1 + (o1 + y)) * g.n2 + (o2 + z)];
    }
    load_halo(g, fb, o0, o1, o2, Hb);
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.y * kT + threadIdx.x;
    if (k >= a.cnt[p]) return;
    const int64_t bi = ((a.auto_mask >> p) & 1) ? k + a.center : k;
    int r0, r1, r2;
    if (g.ndim == 2) {
        r0 = (int)(bi / g.box) - g.P;
        r1 = (int)(bi % g.box) - g.P;
        r2 = 0;
    } else {
        r2 = (int)(bi % g.box) - g.P;
        r1 = (int)((bi / g.box) % g.box) - g.P;
        r0 = (int)(bi / ((int64_t)g.box * g.box)) - g.P;
    }
    const int pz = (g.ndim == 3) ? r2 + g.P : 0;
    double acc = 0.0;
    const float *hb = Hb + ((r0 + g.P) * g.p1 + (r1 + g.P)) * g.h2 + pz;
    if constexpr (TX > 0) {
#pragma unroll
        for (int x = 0; x < TX; ++x) {
            float slab = 0.f;
            // tile row x, the same for every lane: four values per LDS read (the tile
            // starts the block's LDS, and a row is a multiple of 16 floats)
            float av[TY * TZ];
#pragma unroll
            for (int i = 0; i < TY * TZ / 4; ++i) {
                const float4 v4 = reinterpret_cast<const float4 *>(Ta + x * TY * TZ)[i];
                av[4 * i] = v4.x;
                av[4 * i + 1] = v4.y;
                av[4 * i + 2] = v4.z;
                av[4 * i + 3] = v4.w;
            }
#pragma unroll
            for (int y = 0; y < TY; ++y) {
                // 2-D (TZ = 1): h2 = 1, so the row offsets are constants the LDS reads carry
                const float *brow = hb + (TZ == 1 ? x * g.p1 + y : (x * g.p1 + y) * g.h2);
#pragma unroll
                for (int z = 0; z < TZ; ++z) slab += pair_term<SOFT>(av[y * TZ + z], brow[z], a.soft);
            }
            acc += (double)slab;
        }
    } else {
        for (int x = 0; x < g.t0; ++x) {
            float slab = 0.f;
            for (int y = 0; y < g.t1; ++y) {
                const float *arow = Ta + (x * g.t1 + y) * g.t2;
                const float *brow = hb + (x * g.p1 + y) * g.h2;
                for (int z = 0; z < g.t2; ++z) slab += pair_term<SOFT>(arow[z], brow[z], a.soft);
            }
            acc += (double)slab;
        }
    }
    a.part[((int64_t)bp * a.ntiles + tile) * a.kmax + k] = acc;
}

struct DirRedArgs {
    const double *part;
    float *S;
    int npairs;
    int64_t ntiles, kmax, K;
    int64_t cnt[kMaxPairs], off[kMaxPairs];
    double invN;
};

// One block per (32 consecutive displacements, batch x pair): lane group q of
// 32 sums tiles q, q + 32, ... in order, eight loads in flight at a time
// (coalesced: the 32 displacements of a tile are contiguous), then the 32 group
// sums are added in group order.  A level's few blocks sit between its forward
// and the error, so each thread has only a few partials to add.
constexpr int kRedK = 32, kRedG = 32, kRedT = kRedK * kRedG;

__global__ __launch_bounds__(kRedT) void k_direct_reduce(DirRedArgs a)
{
    __shared__ double part[kRedG][kRedK];
    const int kk = threadIdx.x % kRedK, grp = threadIdx.x / kRedK;
    const int64_t k = (int64_t)blockIdx.x * kRedK + kk;
    const int bp = blockIdx.y;
    const int p = bp % a.npairs;
    const int64_t b = bp / a.npairs;
    double s = 0.0;
    if (k < a.cnt[p]) {
        const double *src = a.part + (int64_t)bp * a.ntiles * a.kmax + k;
        for (int64_t t0 = grp; t0 < a.ntiles; t0 += 8 * kRedG) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t t = t0 + (int64_t)u * kRedG;
                v[u] = t < a.ntiles ? src[t * a.kmax] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
    }
    part[grp][kk] = s;
    __syncthreads();
    if (grp == 0 && k < a.cnt[p]) {
        double tot = part[0][kk];
        for (int q = 1; q < kRedG; ++q) tot += part[q][kk];
        a.S[b * a.K + a.off[p] + k] = (float)(tot * a.invN);
    }
}

struct DirAdjArgs {
    Soft soft;
    Geo g;
    const float *phi;
    const float *KB0;   // [B][C][C][box^d]
    float *grad;        // [B][C][n..]
    int C;
    int64_t N, vol;
    float invN;
};

// derivative of the pair term with respect to the thread's own end value, up to
// the constant c1 alpha (applied once to the voxel's sum): f(u) sigma (1 - sigma).
// ownk = k1 own + k0, formed once per voxel.
template <bool SOFT>
__device__ __forceinline__ float adj_term(float ownk, float other, const Soft &s)
{
    if constexpr (SOFT) {
        const float sg = soft_sigma2(fmaf(other, s.k1, ownk));
        return fmaf(s.c1, sg, s.c3) * fmaf(-sg, sg, sg);
    } else {
        return other;
    }
}

// The adjoint has one output per voxel but |box| terms each: adj_split threads
// share a voxel, each taking every adj_split-th box row r0; the partial sums are
// added in split order.  The soft term (exp and reciprocal) is bound by issue and
// takes four shares, so that a tile of 256 voxels keeps 16 waves busy; the product
// term is one multiply-add, and two shares spread the block's set-up (halo load,
// index and address arithmetic) over twice the terms.
constexpr int kAdjSplit = 4;   // the most shares any variant takes (LDS budget)
template <bool SOFT>
constexpr int adj_split()
{
    return SOFT ? 4 : 2;
}

template <bool SOFT>
__global__ __launch_bounds__(kT * adj_split<SOFT>()) void k_direct_adj(DirAdjArgs a)
{
    constexpr int kSplit = adj_split<SOFT>();
    constexpr int kAdjT = kT * kSplit;
    extern __shared__ float sm[];
    const Geo &g = a.g;
    const int tile = blockIdx.x;
    const int c = blockIdx.y;
    const int64_t b = blockIdx.z;
    int tx, ty, tz;
    split3(tile, g.nt1, g.nt2, g.ndim == 2, tx, ty, tz);
    const int o0 = tx * g.t0, o1 = ty * g.t1, o2 = tz * g.t2;
    const int tvol = g.t0 * g.t1 * g.t2;
    const int hvol = g.h0 * g.p1 * g.h2;
    float *red = sm + hvol;            // [kSplit][kT] partial sums
    // this thread's output voxel and its share of the box rows; kT is a multiple of
    // the wave size, so split is the same in every lane of a wave, and saying so lets
    // the kernel rows be read by scalar loads instead of a vector load per term
    static_assert(kT % 64 == 0, "a wave must not straddle two row shares");
    const int v = threadIdx.x % kT, split = __builtin_amdgcn_readfirstlane(threadIdx.x / kT);
    int vx, vy, vz;
    split3(v, g.t1, g.t2, g.ndim == 2, vx, vy, vz);
    const bool active = v < tvol;
    const int64_t vox = ((int64_t)(o0 + vx) * g.n1 + (o1 + vy)) * g.n2 + (o2 + vz);
    // own value phi_c(x), needed by the soft pair term
    const float own = (SOFT && active) ? a.phi[(b * a.C + c) * a.N + vox] : 0.f;
    const float ownk = SOFT ? fmaf(own, a.soft.k1, a.soft.k0) : 0.f;
    float acc = 0.f;
    for (int j = 0; j < a.C; ++j) {
        load_halo<kAdjT>(g, a.phi + (b * a.C + j) * a.N, o0, o1, o2, sm);
        __syncthreads();
        if (active) {
            const float *Kc = a.KB0 + ((b * a.C + c) * a.C + j) * a.vol;
            // the product term's loop is bound by its scalar loop and address work:
            // sixteen terms per step halve it; the soft term keeps eight (long rows
            // would leave a long one-term remainder)
            constexpr int kU = SOFT ? 8 : 16;
            if (g.ndim == 2) {
                for (int r0 = split; r0 < g.box; r0 += kSplit) {
                    const float *hrow = sm + (vx + r0) * g.p1 + vy;
                    const float *krow = Kc + r0 * g.box;
#pragma unroll kU
                    for (int r1 = 0; r1 < g.box; ++r1) acc += krow[r1] * adj_term<SOFT>(ownk, hrow[r1], a.soft);
                }
            } else {
                for (int r0 = split; r0 < g.box; r0 += kSplit)
                    for (int r1 = 0; r1 < g.box; ++r1) {
                        const float *hrow = sm + ((vx + r0) * g.p1 + (vy + r1)) * g.h2 + vz;
                        const float *krow = Kc + (r0 * g.box + r1) * g.box;
#pragma unroll kU
                        for (int r2 = 0; r2 < g.box; ++r2) acc += krow[r2] * adj_term<SOFT>(ownk, hrow[r2], a.soft);
                    }
            }
        }
        __syncthreads();
    }
    red[split * kT + v] = acc;
    __syncthreads();
    if (split == 0 && active) {
        float t = red[v];
#pragma unroll
        for (int q = 1; q < kSplit; ++q) t += red[q * kT + v];
        a.grad[(b * a.C + c) * a.N + vox] = t * (SOFT ? a.soft.c1a : 1.f) * a.invN;
    }
}

Soft make_soft(const Plan &p)
{
    const double log2e = 1.4426950408889634074;
    return Soft{(float)(-0.5 * p.alpha * log2e), (float)(-p.alpha * p.c2 * log2e), (float)p.c1, (float)p.c3,
                (float)(p.c1 * p.alpha)};
}

// LDS pitch of the halo's axis-1 rows for tile t at displacement range P.  In
// 2-D a wave of the adjoint reads four tile rows of 16 voxels (two per
// half-wave), one row pitch apart: a pitch of 16 mod 32 floats puts the two rows
// of a half-wave in disjoint banks of the 32, where a pitch of 32 (P = 8) or 64
// (P = 24) puts them in the same banks.  The padded pitch is taken where the
// padded halo still fits the LDS budget, else the plain one (which decides
// support).  The 3-D tile's wave reads rows h2 apart within one plane and keeps
// the plain pitch.
int halo_pitch1(int ndim, const int t[3], int P)
{
    const int64_t h0 = t[0] + 2 * P, h1 = t[1] + 2 * P, h2 = ndim == 3 ? t[2] + 2 * P : 1;
    if (ndim != 2) return (int)h1;
    const int64_t pad = h1 + (48 - h1 % 32) % 32;
    const int64_t tvol = (int64_t)t[0] * t[1] * t[2];
    const int64_t extra = tvol > (int64_t)kAdjSplit * kT ? tvol : (int64_t)kAdjSplit * kT;
    return (size_t)(extra + h0 * pad * h2) * sizeof(float) <= kDirectLds ? (int)pad : (int)h1;
}

Geo make_geo(const Plan &p, int l)
{
    const LevelPlan &L = p.lv[l];
    Geo g{};
    g.ndim = p.ndim;
    g.n0 = L.n[0];
    g.n1 = L.n[1];
    g.n2 = p.ndim == 3 ? L.n[2] : 1;
    g.t0 = L.tile[0];
    g.t1 = L.tile[1];
    g.t2 = L.tile[2];
    g.P = L.P;
    g.box = L.box;
    g.h0 = g.t0 + 2 * L.P;
    g.h1 = g.t1 + 2 * L.P;
    g.h2 = p.ndim == 3 ? g.t2 + 2 * L.P : 1;
    g.p1 = halo_pitch1(p.ndim, L.tile, L.P);
    g.nt0 = g.n0 / g.t0;
    g.nt1 = g.n1 / g.t1;
    g.nt2 = g.n2 / g.t2;
    return g;
}

}  // namespace

bool direct_supported(const Plan &p, int l, int tile[3])
{
    const LevelPlan &L = p.lv[l];
    // tiles of 256 voxels: 16 x 16 in 2-D, 4 x 8 x 8 in 3-D (clipped to the grid)
    int t[3];
    if (p.ndim == 2) {
        t[0] = L.n[0] < 16 ? L.n[0] : 16;
        t[1] = L.n[1] < 16 ? L.n[1] : 16;
        t[2] = 1;
    } else {
        t[0] = L.n[0] < 4 ? L.n[0] : 4;
        t[1] = L.n[1] < 8 ? L.n[1] : 8;
        t[2] = L.n[2] < 8 ? L.n[2] : 8;
    }
    const int64_t tvol = (int64_t)t[0] * t[1] * t[2];
    int64_t hvol = (int64_t)(t[0] + 2 * L.P) * (t[1] + 2 * L.P);
    if (p.ndim == 3) hvol *= (t[2] + 2 * L.P);
    // forward: tile + halo; adjoint: halo + the kAdjSplit x 256 partial sums
    const int64_t extra = tvol > (int64_t)kAdjSplit * kT ? tvol : (int64_t)kAdjSplit * kT;
    if ((size_t)(extra + hvol) * sizeof(float) > kDirectLds) return false;
    if (tile) {
        tile[0] = t[0];
        tile[1] = t[1];
        tile[2] = t[2];
    }
    return true;
}

hipError_t direct_forward_level(const Plan &p, int l, const float *phi, float *S, const Ws &ws,
                                hipStream_t st)
{
    const LevelPlan &L = p.lv[l];
    DirFwdArgs a{};
    a.soft = make_soft(p);
    a.g = make_geo(p, l);
    a.phi = phi;
    a.part = ws.at<double>(L.part);
    a.C = p.C;
    a.npairs = p.npairs;
    a.N = L.N;
    a.ntiles = L.n_tiles;
    int64_t kmax = 0, vol = 1;
    for (int d = 0; d < p.ndim; ++d) vol *= L.box;
    a.center = (vol - 1) / 2;
    for (int q = 0; q < p.npairs; ++q) {
        a.pi[q] = p.pi[q];
        a.pj[q] = p.pj[q];
        if (p.pi[q] == p.pj[q]) a.auto_mask |= 1 << q;
        a.cnt[q] = L.cnt[q];
        if (L.cnt[q] > kmax) kmax = L.cnt[q];
    }
    a.kmax = kmax;
    const int tvol = a.g.t0 * a.g.t1 * a.g.t2;
    const size_t lds = (size_t)(tvol + a.g.h0 * a.g.p1 * a.g.h2) * sizeof(float);
    dim3 grid((unsigned)a.ntiles, (unsigned)((kmax + kT - 1) / kT), (unsigned)(p.B * p.npairs));
    const double fbytes = (double)p.B * p.C * L.N * 4 + (double)p.B * p.npairs * a.ntiles * kmax * 8;
    const bool full2 = p.ndim == 2 && a.g.t0 == 16 && a.g.t1 == 16;
    const bool full3 = p.ndim == 3 && a.g.t0 == 4 && a.g.t1 == 8 && a.g.t2 == 8;
    const bool soft = p.desc != DMCR_DESC_S2;
    const char *name = soft ? "direct_fwd_soft" : "direct_fwd";
    hipError_t e;
    if (full2)
        e = soft ? launch(name, fbytes, k_direct_fwd<true, 16, 16, 1>, grid, dim3(kT), lds, st, a)
                 : launch(name, fbytes, k_direct_fwd<false, 16, 16, 1>, grid, dim3(kT), lds, st, a);
    else if (full3)
        e = soft ? launch(name, fbytes, k_direct_fwd<true, 4, 8, 8>, grid, dim3(kT), lds, st, a)
                 : launch(name, fbytes, k_direct_fwd<false, 4, 8, 8>, grid, dim3(kT), lds, st, a);
    else
        e = soft ? launch(name, fbytes, k_direct_fwd<true, 0, 0, 0>, grid, dim3(kT), lds, st, a)
                 : launch(name, fbytes, k_direct_fwd<false, 0, 0, 0>, grid, dim3(kT), lds, st, a);
    if (e != hipSuccess) return e;
    DirRedArgs r{};
    r.part = a.part;
    r.S = S;
    r.npairs = p.npairs;
    r.ntiles = a.ntiles;
    r.kmax = kmax;
    r.K = p.K;
    for (int q = 0; q < p.npairs; ++q) {
        r.cnt[q] = L.cnt[q];
        r.off[q] = L.off[q];
    }
    r.invN = 1.0 / (double)L.N;
    dim3 rg((unsigned)((kmax + kRedK - 1) / kRedK), (unsigned)(p.B * p.npairs));
    return launch("direct_reduce", (double)p.B * p.npairs * a.ntiles * kmax * 8, k_direct_reduce, rg, dim3(kRedT), 0,
                  st, r);
}

hipError_t direct_adjoint_level(const Plan &p, int l, const float *phi, const float *G, float *grad,
                                const Ws &ws, hipStream_t st, const double *St)
{
    const LevelPlan &L = p.lv[l];
    float *KB0 = ws.at<float>(L.KB0);
    hipError_t e = launch_build_kernels(p, l, G, KB0, st, St);
    if (e != hipSuccess) return e;
    DirAdjArgs a{};
    a.soft = make_soft(p);
    a.g = make_geo(p, l);
    a.phi = phi;
    a.KB0 = KB0;
    a.grad = grad;
    a.C = p.C;
    a.N = L.N;
    a.vol = 1;
    for (int d = 0; d < p.ndim; ++d) a.vol *= L.box;
    a.invN = (float)(1.0 / (double)L.N);
    const size_t lds = (size_t)(a.g.h0 * a.g.p1 * a.g.h2 + kAdjSplit * kT) * sizeof(float);
    dim3 grid((unsigned)L.n_tiles, (unsigned)p.C, (unsigned)p.B);
    const double bytes = 2.0 * p.B * p.C * L.N * 4 + (double)p.B * p.C * p.C * a.vol * 4;
    if (p.desc == DMCR_DESC_S2)
        return launch("direct_adj", bytes, k_direct_adj<false>, grid, dim3(kT * adj_split<false>()), lds, st, a);
    return launch("direct_adj_soft", bytes, k_direct_adj<true>, grid, dim3(kT * adj_split<true>()), lds, st, a);
}

}  // namespace dmcr
