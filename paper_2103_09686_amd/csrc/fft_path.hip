// FFT path of the descriptor: S_ij = (1/N^2) IDFT(conj(DFT phi_i) DFT phi_j) on the
// displacement box, and its adjoint grad_c = (1/N^2) IDFT(sum_j conj(DFT K_cj) DFT phi_j)
// where K_cj are the cotangents laid out on the box (see build_kernels.hip).
//
// This replaces the paper's dense mask convolution (Sec. 3.2.3, eq. convdef;
// Appendix B) by the convolution theorem, which the paper names as the
// Fourier route to correlations (Sec. 3.2, Sec. 3.4.1).  The transform along
// the contiguous axis is real-to-half-complex; the other axes are complex.
// Transforms are pruned: the inverse keeps only rows |r| <= P of each axis,
// and the transforms of the cotangent boxes read only those rows.
//
// Kernels (all one pass over HBM, work staged in LDS):
//   k_pass       generic 1-D transform of a batch of pencils along one axis
//   k_axis0_fwd  axis-0 forward DFT of every channel, pair products, pruned
//                axis-0 inverse (the "reduce" step fused into the transform)
//   k_axis0_adj  axis-0 forward DFT of fields and cotangent boxes, the adjoint
//                product sum, full axis-0 inverse (in place)
#include "dmcr_internal.h"
#include "lds_fft.h"

namespace dmcr {

namespace {

__device__ __forceinline__ int wrap_box(int e, int P, int n)
{
    int pos = e - P;
    return pos < 0 ? pos + n : pos;
}

struct PassArgs {
    const void *in;
    void *out;
    int64_t npen;     // number of pencils
    int64_t inner;    // element stride along the transformed axis
    int n, log2n, T;  // transform length, pencils per block
    int in_mode, out_mode;
    int in_len, out_len;  // rows of the input / output arrays along the axis
    int P;
    int in_real, out_real, inv;
    float scale;
    // IO_DESC: pencil m = (b * npairs + p) * rows_per_pair + row; entry e of the
    // row is box index row * box + e of pair p.
    int npairs, auto_mask;
    int64_t rows_per_pair, center, Kstride;
    int64_t off[kMaxPairs];
};

__global__ __launch_bounds__(NT) void k_pass(PassArgs a)
{
    extern __shared__ float2 sm[];
    const int n = a.n, T = a.T;
    float2 *tw = sm;
    float2 *buf = sm + n;
    const int64_t m0 = (int64_t)blockIdx.x * T;
    init_twiddles(tw, n);
    if (a.in_mode == IO_BOX) {
        for (int i = threadIdx.x; i < T * n; i += NT) buf[i] = make_float2(0.f, 0.f);
        __syncthreads();
    }
    const int total_in = T * a.in_len;
    for (int idx = threadIdx.x; idx < total_in; idx += NT) {
        int t, e;
        if (a.inner == 1) {
            t = idx / a.in_len;
            e = idx - t * a.in_len;
        } else {
            e = idx / T;
            t = idx - e * T;
        }
        const int64_t m = m0 + t;
        float2 v = make_float2(0.f, 0.f);
        if (m < a.npen) {
            const int64_t o = m / a.inner;
            const int64_t i = m - o * a.inner;
            const int64_t addr = (o * a.in_len + e) * a.inner + i;
            if (a.in_real)
                v.x = static_cast<const float *>(a.in)[addr];
            else
                v = static_cast<const float2 *>(a.in)[addr];
        }
        const int pos = (a.in_mode == IO_BOX) ? wrap_box(e, a.P, n) : e;
        buf[pos * T + t] = v;
        if (a.in_mode == IO_HALF && e > 0 && e < n / 2) buf[(n - e) * T + t] = c_conj(v);
    }
    __syncthreads();
    lds_fft(buf, T, T, n, a.log2n, tw, a.inv != 0);
    const int total_out = T * a.out_len;
    for (int idx = threadIdx.x; idx < total_out; idx += NT) {
        int t, e;
        if (a.inner == 1) {
            t = idx / a.out_len;
            e = idx - t * a.out_len;
        } else {
            e = idx / T;
            t = idx - e * T;
        }
        const int64_t m = m0 + t;
        if (m >= a.npen) continue;
        const int pos = (a.out_mode == IO_BOX || a.out_mode == IO_DESC) ? wrap_box(e, a.P, n) : e;
        const float2 v = c_scale(buf[pos * T + t], a.scale);
        if (a.out_mode == IO_DESC) {
            const int64_t row = m % a.rows_per_pair;
            const int64_t bp = m / a.rows_per_pair;
            const int p = (int)(bp % a.npairs);
            const int64_t b = bp / a.npairs;
            const int64_t bi = row * a.out_len + e;
            int64_t k = bi;
            if ((a.auto_mask >> p) & 1) {
                if (bi < a.center) continue;
                k = bi - a.center;
            }
            static_cast<float *>(a.out)[b * a.Kstride + a.off[p] + k] = v.x;
        } else {
            const int64_t o = m / a.inner;
            const int64_t i = m - o * a.inner;
            const int64_t addr = (o * a.out_len + e) * a.inner + i;
            if (a.out_real)
                static_cast<float *>(a.out)[addr] = v.x;
            else
                static_cast<float2 *>(a.out)[addr] = v;
        }
    }
}

struct Axis0Args {
    float2 *X;          // [B][C][n][inner] partial spectra (axes 1.. transformed)
    const float2 *KB;   // adjoint: [B][C*C][box][inner]
    float2 *Y;          // forward: [B][npairs][box][inner]
    int64_t inner, nloc;  // nloc = B * inner pencil locations
    int C, n, log2n, P, box, T, npairs;
    int pi[kMaxPairs], pj[kMaxPairs];
    float scale;
};

// Load the axis-0 pencils of every channel at T consecutive locations into
// A[e * (C*T) + c*T + t].
__device__ __forceinline__ void load_channels(const Axis0Args &a, int64_t m0, float2 *A)
{
    const int CT = a.C * a.T;
    const int total = CT * a.n;
    for (int idx = threadIdx.x; idx < total; idx += NT) {
        const int t = idx % a.T;
        const int r = idx / a.T;
        const int c = r % a.C;
        const int e = r / a.C;
        const int64_t m = m0 + t;
        float2 v = make_float2(0.f, 0.f);
        if (m < a.nloc) {
            const int64_t b = m / a.inner;
            const int64_t i = m - b * a.inner;
            v = a.X[((b * a.C + c) * a.n + e) * a.inner + i];
        }
        A[e * CT + c * a.T + t] = v;
    }
}

__global__ __launch_bounds__(NT) void k_axis0_fwd(Axis0Args a)
{
    extern __shared__ float2 sm[];
    const int n = a.n, T = a.T, CT = a.C * a.T;
    float2 *tw = sm;
    float2 *A = tw + n;
    float2 *W = A + CT * n;
    const int64_t m0 = (int64_t)blockIdx.x * T;
    init_twiddles(tw, n);
    load_channels(a, m0, A);
    __syncthreads();
    lds_fft(A, CT, CT, n, a.log2n, tw, false);
    for (int p = 0; p < a.npairs; ++p) {
        const int ci = a.pi[p], cj = a.pj[p];
        for (int idx = threadIdx.x; idx < T * n; idx += NT) {
            const int e = idx / T, t = idx - e * T;
            W[idx] = c_scale(c_cmul(A[e * CT + ci * T + t], A[e * CT + cj * T + t]), a.scale);
        }
        __syncthreads();
        lds_fft(W, T, T, n, a.log2n, tw, true);
        for (int idx = threadIdx.x; idx < T * a.box; idx += NT) {
            const int e = idx / T, t = idx - e * T;
            const int64_t m = m0 + t;
            if (m < a.nloc) {
                const int64_t b = m / a.inner;
                const int64_t i = m - b * a.inner;
                a.Y[((b * a.npairs + p) * a.box + e) * a.inner + i] = W[wrap_box(e, a.P, n) * T + t];
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(NT) void k_axis0_adj(Axis0Args a)
{
    extern __shared__ float2 sm[];
    const int n = a.n, T = a.T, C = a.C, CT = a.C * a.T;
    float2 *tw = sm;
    float2 *A = tw + n;
    float2 *W = A + CT * n;
    float2 *ACC = W + CT * n;
    const int64_t m0 = (int64_t)blockIdx.x * T;
    init_twiddles(tw, n);
    load_channels(a, m0, A);
    __syncthreads();
    lds_fft(A, CT, CT, n, a.log2n, tw, false);
    for (int c = 0; c < C; ++c) {
        for (int i = threadIdx.x; i < CT * n; i += NT) W[i] = make_float2(0.f, 0.f);
        __syncthreads();
        for (int idx = threadIdx.x; idx < CT * a.box; idx += NT) {
            const int t = idx % T;
            const int r = idx / T;
            const int j = r % C;
            const int e = r / C;
            const int64_t m = m0 + t;
            if (m < a.nloc) {
                const int64_t b = m / a.inner;
                const int64_t i = m - b * a.inner;
                W[wrap_box(e, a.P, n) * CT + j * T + t] =
                    a.KB[((b * C * C + c * C + j) * a.box + e) * a.inner + i];
            }
        }
        __syncthreads();
        lds_fft(W, CT, CT, n, a.log2n, tw, false);
        for (int idx = threadIdx.x; idx < T * n; idx += NT) {
            const int e = idx / T, t = idx - e * T;
            float2 s = make_float2(0.f, 0.f);
            for (int j = 0; j < C; ++j)
                s = c_add(s, c_cmul(W[e * CT + j * T + t], A[e * CT + j * T + t]));
            ACC[idx] = c_scale(s, a.scale);
        }
        __syncthreads();
        lds_fft(ACC, T, T, n, a.log2n, tw, true);
        for (int idx = threadIdx.x; idx < T * n; idx += NT) {
            const int e = idx / T, t = idx - e * T;
            const int64_t m = m0 + t;
            if (m < a.nloc) {
                const int64_t b = m / a.inner;
                const int64_t i = m - b * a.inner;
                a.X[((b * C + c) * n + e) * a.inner + i] = ACC[idx];
            }
        }
        __syncthreads();
    }
}

int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

int pow2_floor(int x)
{
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

constexpr size_t kLdsBudget = 64 * 1024;  // bytes of dynamic LDS per block

hipError_t run_pass(PassArgs a, hipStream_t st)
{
    // pencils per block: fill the FFT budget, at most 64 pencils
    int T = kFftMaxElems / a.n;
    T = T > 64 ? 64 : T;
    while (T > 1 && (size_t)(a.n + T * a.n) * sizeof(float2) > kLdsBudget) T /= 2;
    if (T < 1) T = 1;
    if ((int64_t)T > a.npen) T = pow2_floor((int)(a.npen < 1 ? 1 : a.npen));
    a.T = T;
    a.log2n = ilog2(a.n);
    const int64_t blocks = (a.npen + T - 1) / T;
    const size_t lds = (size_t)(a.n + T * a.n) * sizeof(float2);
    hipLaunchKernelGGL(k_pass, dim3((unsigned)blocks), dim3(NT), lds, st, a);
    return hipGetLastError();
}

PassArgs pass_args(const void *in, void *out, int64_t npen, int64_t inner, int n, int in_mode,
                   int in_len, int out_mode, int out_len, int P, bool in_real, bool out_real, bool inv,
                   float scale)
{
    PassArgs a{};
    a.in = in;
    a.out = out;
    a.npen = npen;
    a.inner = inner;
    a.n = n;
    a.in_mode = in_mode;
    a.in_len = in_len;
    a.out_mode = out_mode;
    a.out_len = out_len;
    a.P = P;
    a.in_real = in_real;
    a.out_real = out_real;
    a.inv = inv;
    a.scale = scale;
    return a;
}

int axis0_T(int C, int n, int bufs_of_CT, int extra)
{
    // LDS = (n + (bufs_of_CT*C + extra) * T * n) * 8 <= budget; FFT call C*T*n <= max
    int T = 16;
    while (T > 1 && ((size_t)(n + (bufs_of_CT * C + extra) * T * n) * sizeof(float2) > kLdsBudget ||
                     C * T * n > kFftMaxElems))
        T /= 2;
    return T;
}

}  // namespace

bool fft_supported(const Plan &p, int l)
{
    const LevelPlan &L = p.lv[l];
    for (int a = 0; a < p.ndim; ++a)
        if (L.n[a] > kMaxFft || L.n[a] < 2) return false;
    const int n0 = L.n[0];
    const int C = p.C;
    // axis-0 adjoint kernel needs (2C + 1) T n0 + n0 complex values with T >= 1
    if ((size_t)(n0 + (2 * C + 1) * n0) * sizeof(float2) > kLdsBudget) return false;
    if (C * n0 > kFftMaxElems) return false;
    return true;
}

// Half spectrum of every channel, transformed along every axis except 0:
// X = DFT_{1..d-1}(phi) (the contiguous axis real-to-half-complex).
hipError_t fft_spectrum_level(const Plan &p, int l, const float *phi, const Ws &ws, hipStream_t st)
{
    const LevelPlan &L = p.lv[l];
    const int B = p.B, C = p.C;
    float2 *X = ws.at<float2>(L.X);
    hipError_t e;
    if (p.ndim == 2) {
        const int n0 = L.n[0], n1 = L.n[1];
        e = run_pass(pass_args(phi, X, (int64_t)B * C * n0, 1, n1, IO_FULL, n1, IO_HALF, L.h, 0, true,
                               false, false, 1.f), st);
        return e;
    }
    const int n0 = L.n[0], n1 = L.n[1], n2 = L.n[2];
    e = run_pass(pass_args(phi, X, (int64_t)B * C * n0 * n1, 1, n2, IO_FULL, n2, IO_HALF, L.h, 0, true,
                           false, false, 1.f), st);
    if (e != hipSuccess) return e;
    e = run_pass(pass_args(X, X, (int64_t)B * C * n0 * L.h, L.h, n1, IO_FULL, n1, IO_FULL, n1, 0, false,
                           false, false, 1.f), st);
    return e;
}

hipError_t fft_forward_level(const Plan &p, int l, const float *phi, float *S, const Ws &ws,
                             hipStream_t st)
{
    const LevelPlan &L = p.lv[l];
    const int B = p.B, C = p.C;
    hipError_t e = fft_spectrum_level(p, l, phi, ws, st);
    if (e != hipSuccess) return e;
    float2 *X = ws.at<float2>(L.X);
    float2 *Y = ws.at<float2>(L.Y);
    const int n0 = L.n[0];
    const int64_t inner = (p.ndim == 2) ? L.h : (int64_t)L.n[1] * L.h;
    const double invN = 1.0 / (double)L.N;

    Axis0Args a{};
    a.X = X;
    a.Y = Y;
    a.inner = inner;
    a.nloc = (int64_t)B * inner;
    a.C = C;
    a.n = n0;
    a.log2n = ilog2(n0);
    a.P = L.P;
    a.box = L.box;
    a.npairs = p.npairs;
    for (int q = 0; q < p.npairs; ++q) {
        a.pi[q] = p.pi[q];
        a.pj[q] = p.pj[q];
    }
    a.scale = (float)(invN * invN);
    a.T = axis0_T(C, n0, 1, 1);
    {
        const size_t lds = (size_t)(n0 + (C + 1) * a.T * n0) * sizeof(float2);
        const int64_t blocks = (a.nloc + a.T - 1) / a.T;
        hipLaunchKernelGGL(k_axis0_fwd, dim3((unsigned)blocks), dim3(NT), lds, st, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }

    // remaining inverse axes, pruned, then scatter into descriptor order
    const float2 *last_in = Y;
    int64_t rows_per_pair = L.box;
    if (p.ndim == 3) {
        float2 *Y2 = ws.at<float2>(L.Y2);
        e = run_pass(pass_args(Y, Y2, (int64_t)B * p.npairs * L.box * L.h, L.h, L.n[1], IO_FULL, L.n[1],
                               IO_BOX, L.box, L.P, false, false, true, 1.f), st);
        if (e != hipSuccess) return e;
        last_in = Y2;
        rows_per_pair = (int64_t)L.box * L.box;
    }
    const int nl = L.n[p.ndim - 1];
    PassArgs d = pass_args(last_in, S + 0, (int64_t)B * p.npairs * rows_per_pair, 1, nl, IO_HALF, L.h,
                           IO_DESC, L.box, L.P, false, true, true, 1.f);
    d.npairs = p.npairs;
    d.rows_per_pair = rows_per_pair;
    d.Kstride = p.K;
    int64_t boxvol = 1;
    for (int a2 = 0; a2 < p.ndim; ++a2) boxvol *= L.box;
    d.center = (boxvol - 1) / 2;
    d.auto_mask = 0;
    for (int q = 0; q < p.npairs; ++q) {
        d.off[q] = L.off[q];
        if (p.pi[q] == p.pj[q]) d.auto_mask |= 1 << q;
    }
    return run_pass(d, st);
}

hipError_t fft_adjoint_level(const Plan &p, int l, const float *phi, const float *G, float *grad,
                             bool have_spectrum, const Ws &ws, hipStream_t st)
{
    const LevelPlan &L = p.lv[l];
    const int B = p.B, C = p.C, CC = C * C;
    hipError_t e;
    float *KB0 = ws.at<float>(L.KB0);
    float2 *KB1 = ws.at<float2>(L.KB1);
    e = launch_build_kernels(p, l, G, KB0, st);
    if (e != hipSuccess) return e;
    const int nl = L.n[p.ndim - 1];
    const float2 *KBaxis0;
    if (p.ndim == 2) {
        e = run_pass(pass_args(KB0, KB1, (int64_t)B * CC * L.box, 1, nl, IO_BOX, L.box, IO_HALF, L.h, L.P,
                               true, false, false, 1.f), st);
        if (e != hipSuccess) return e;
        KBaxis0 = KB1;
    } else {
        float2 *KB2 = ws.at<float2>(L.KB2);
        e = run_pass(pass_args(KB0, KB1, (int64_t)B * CC * L.box * L.box, 1, nl, IO_BOX, L.box, IO_HALF,
                               L.h, L.P, true, false, false, 1.f), st);
        if (e != hipSuccess) return e;
        e = run_pass(pass_args(KB1, KB2, (int64_t)B * CC * L.box * L.h, L.h, L.n[1], IO_BOX, L.box, IO_FULL,
                               L.n[1], L.P, false, false, false, 1.f), st);
        if (e != hipSuccess) return e;
        KBaxis0 = KB2;
    }
    if (!have_spectrum) {
        e = fft_spectrum_level(p, l, phi, ws, st);
        if (e != hipSuccess) return e;
    }
    float2 *X = ws.at<float2>(L.X);
    const int n0 = L.n[0];
    const int64_t inner = (p.ndim == 2) ? L.h : (int64_t)L.n[1] * L.h;
    const double invN = 1.0 / (double)L.N;
    Axis0Args a{};
    a.X = X;
    a.KB = KBaxis0;
    a.inner = inner;
    a.nloc = (int64_t)B * inner;
    a.C = C;
    a.n = n0;
    a.log2n = ilog2(n0);
    a.P = L.P;
    a.box = L.box;
    a.scale = (float)(invN * invN);
    a.T = axis0_T(C, n0, 2, 1);
    {
        const size_t lds = (size_t)(n0 + (2 * C + 1) * a.T * n0) * sizeof(float2);
        const int64_t blocks = (a.nloc + a.T - 1) / a.T;
        hipLaunchKernelGGL(k_axis0_adj, dim3((unsigned)blocks), dim3(NT), lds, st, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (p.ndim == 3) {
        e = run_pass(pass_args(X, X, (int64_t)B * C * n0 * L.h, L.h, L.n[1], IO_FULL, L.n[1], IO_FULL, L.n[1],
                               0, false, false, true, 1.f), st);
        if (e != hipSuccess) return e;
    }
    const int64_t rows = (p.ndim == 2) ? (int64_t)B * C * n0 : (int64_t)B * C * n0 * L.n[1];
    return run_pass(pass_args(X, grad, rows, 1, nl, IO_HALF, L.h, IO_FULL, nl, 0, false, true, true, 1.f),
                    st);
}

}  // namespace dmcr
