// Radix-4/2 Stockham FFT on pencils held in LDS, for gfx950 (wave64).
//
// A block of NT threads transforms `npen` independent pencils of length n
// (a power of two, 1..1024).  Element e of pencil t lives at buf[e*ps + t],
// so consecutive lanes touch consecutive pencils and the LDS accesses of a
// stage are unit-stride across a wave.  Each stage reads its inputs into
// registers, synchronises, and writes the sorted outputs back in place
// (Stockham auto-sort: no bit reversal pass).  Twiddles come from an LDS table
// tw[m] = exp(-2 pi i m / n), computed in float64 and rounded once.
//
// The stage structure (span Ns, butterfly j, twiddle exponent q*(j mod Ns),
// output slot (j div Ns)*Ns*R + j mod Ns + q*Ns) is the standard
// out-of-place Stockham formulation for GPUs (Govindaraju et al., SC'08).
#pragma once

#include <hip/hip_runtime.h>

namespace dmcr {

constexpr int NT = 256;         // threads per block of every FFT kernel
constexpr int kFftMaxPer = 8;   // radix-4 butterflies per thread per stage
constexpr int kFftMaxElems = NT * kFftMaxPer * 4;  // npen * n limit of one call (8192)

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

// tw[m] = exp(-2 pi i m / n), m < n.  Caller synchronises before use.
__device__ __forceinline__ void init_twiddles(float2 *tw, int n)
{
    for (int m = threadIdx.x; m < n; m += NT) {
        double s, c;
        sincospi(2.0 * (double)m / (double)n, &s, &c);
        tw[m] = make_float2((float)c, (float)(-s));
    }
}

template <int R>
__device__ __forceinline__ void small_dft(float2 (&v)[R], bool inv);

template <>
__device__ __forceinline__ void small_dft<2>(float2 (&v)[2], bool)
{
    const float2 a = v[0], b = v[1];
    v[0] = c_add(a, b);
    v[1] = c_sub(a, b);
}

template <>
__device__ __forceinline__ void small_dft<4>(float2 (&v)[4], bool inv)
{
    const float2 a0 = c_add(v[0], v[2]);
    const float2 a1 = c_sub(v[0], v[2]);
    const float2 a2 = c_add(v[1], v[3]);
    const float2 d = c_sub(v[1], v[3]);
    // d times exp(-+ i pi/2): forward -i*d, inverse +i*d
    const float2 wd = inv ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
    v[0] = c_add(a0, a2);
    v[2] = c_sub(a0, a2);
    v[1] = c_add(a1, wd);
    v[3] = c_sub(a1, wd);
}

template <int R, int MAXPER>
__device__ __forceinline__ void fft_stage(float2 *buf, int ps, int npen, int n, int Ns,
                                          const float2 *tw, bool inv)
{
    const int nb = n / R;
    const int total = npen * nb;
    const int twstep = n / (Ns * R);
    float2 v[MAXPER][R];
#pragma unroll
    for (int i = 0; i < MAXPER; ++i) {
        const int idx = threadIdx.x + i * NT;
        if (idx < total) {
            const int j = idx / npen;
            const int t = idx - j * npen;
            const int k = j & (Ns - 1);
#pragma unroll
            for (int q = 0; q < R; ++q) v[i][q] = buf[(j + q * nb) * ps + t];
            if (Ns > 1) {
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    float2 w = tw[q * k * twstep];
                    if (inv) w.y = -w.y;
                    v[i][q] = c_mul(v[i][q], w);
                }
            }
            small_dft<R>(v[i], inv);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXPER; ++i) {
        const int idx = threadIdx.x + i * NT;
        if (idx < total) {
            const int j = idx / npen;
            const int t = idx - j * npen;
            const int k = j & (Ns - 1);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[(base + q * Ns) * ps + t] = v[i][q];
        }
    }
    __syncthreads();
}

// Unnormalised DFT of every pencil: forward uses exp(-2 pi i ...), inverse
// exp(+2 pi i ...).  Requires npen * n <= kFftMaxElems.  Entry and exit are
// block-synchronised by the caller / the last stage.
__device__ __forceinline__ void lds_fft(float2 *buf, int ps, int npen, int n, int log2n,
                                        const float2 *tw, bool inv)
{
    int Ns = 1;
    if (log2n & 1) {
        fft_stage<2, 2 * kFftMaxPer>(buf, ps, npen, n, 1, tw, inv);
        Ns = 2;
    }
    for (; Ns < n; Ns <<= 2) fft_stage<4, kFftMaxPer>(buf, ps, npen, n, Ns, tw, inv);
}

}  // namespace dmcr
