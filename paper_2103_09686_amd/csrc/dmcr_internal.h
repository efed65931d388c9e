// Internal declarations of libdmcr: the per-call plan and the kernel launchers.
// Not part of the public ABI (include/dmcr.h is).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "../../include/dmcr.h"

namespace dmcr {

constexpr int kMaxLevels = DMCR_MAX_LEVELS;
constexpr int kMaxChannels = DMCR_MAX_CHANNELS;
constexpr int kMaxPairs = DMCR_MAX_PAIRS;
constexpr int kMaxFft = 1024;          // longest axis handled by the LDS transforms
constexpr size_t kAlign = 256;
// field buffers move as float pairs: phi, gradients and pyramid levels need 8-byte alignment
inline bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7) == 0; }

// Rows stored along a transformed axis: all n (FULL), the first n/2+1 of a
// Hermitian half spectrum (HALF), the 2P+1 rows |r| <= P in box order (BOX),
// box rows scattered into descriptor order (DESC), or box rows of the adjoint
// kernels computed on the fly from the cotangent G (GBOX).
enum IoMode { IO_FULL = 0, IO_HALF = 1, IO_BOX = 2, IO_DESC = 3, IO_GBOX = 4 };

struct LevelPlan {
    int n[3];          // level shape; 2-D uses n[0], n[1] and n[2] = 1
    int64_t N;         // voxels per channel
    int P;             // max displacement of this level
    int box;           // 2P + 1
    int path;          // DMCR_PATH_FFT or DMCR_PATH_DIRECT (resolved)
    int h;             // n_last / 2 + 1 (half spectrum along the contiguous axis)
    int hp;            // row pitch of half spectra: h rounded up so that 16-column
                       // tiles of every strided pass start on a 128-byte boundary
    int64_t off[kMaxPairs];   // offset of (level, pair) inside one descriptor
    int64_t cnt[kMaxPairs];   // entries of (level, pair)
    // workspace byte offsets (per call, batch included)
    size_t field;      // level >= 1: pooled field [B][C][n..]
    size_t grad;       // level >= 1: level gradient [B][C][n..]
    size_t X;          // FFT: partial spectrum [B][C][n0][(n1)][h] complex
    size_t Y;          // FFT: after axis-0 inverse, box rows [B][pairs][box][inner]
    size_t Y2;         // FFT 3-D: after axis-1 inverse [B][pairs][box][box][h]
    size_t KB0;        // adjoint kernels on the box, real [B][C*C][box^d]
    size_t KB1;        // after last-axis transform [B][C*C][box^(d-1)][h]
    size_t KB2;        // 3-D: after axis-1 transform [B][C*C][box][n1][h]
    size_t msum;       // FFT: float64 partial sums of every field [B][C][mparts]
    int64_t mparts;    // FFT: partial sums per field (fft_mean_parts)
    size_t mu;         // FFT: float64 field means [B][C]
    size_t part;       // DIRECT: per-tile partial sums (float64)
    int64_t n_tiles;   // DIRECT: tiles per field
    int tile[3];       // DIRECT: tile edge per axis
    // three-point blocks (spec.s3_max_disp > 0)
    int s3P;           // P3 of this level (0: no block)
    int s3M;           // vectors (2 P3 + 1)^d
    int64_t s3K;       // entries per channel block, M (M + 1) / 2
    int64_t s3off;     // descriptor offset of channel 0's block (channel c at s3off + c s3K)
    int s3VB, s3VBa;   // voxels per block of the forward and of the adjoint
    int64_t s3chunks;  // forward blocks per field and channel (N / s3VB)
    int s3mf;          // contractions on matrix cores (else register-blocked FMA)
    int s3bf[3];       // matrix cores: forward voxel box edge per axis (s3VB voxels)
    int s3ba[3];       // matrix cores: adjoint voxel box edge per axis (s3VBa voxels)
    int s3Kp, s3Mp;    // rows and columns of the expanded cotangent
    size_t s3part;     // [B][C][s3chunks][s3K] float partial sums
    size_t s3Q, s3R;   // adjoint: [B][C][M][N] float per-vector terms (R: FMA product form only)
    size_t s3G;        // adjoint: [B][C][s3Kp][s3Mp] full symmetric cotangent, zero padded
};

struct Plan {
    int desc;          // DMCR_DESC_*
    double alpha, c1, c2, c3;   // soft threshold f(u) = c1 / (1 + exp(-alpha (u + c2))) + c3
    double F;          // f(1/2)^2 (Appendix A)
    double fh;         // f(1/2)
    int s3;            // three-point blocks present
    int ndim;
    int shape[3];
    int C;
    int L;
    int npairs;
    int pi[kMaxPairs], pj[kMaxPairs];
    double w[kMaxLevels];
    int flags;
    int64_t K;
    int64_t lvl_off[kMaxLevels + 1];   // descriptor offset of each level
    double Z;
    int B;
    LevelPlan lv[kMaxLevels];
    size_t S;          // float [B][K]
    size_t G;          // float [B][K]
    size_t Epart;      // double [B][err_chunks]
    int64_t err_chunks;
    size_t Pen;        // double [B][pen_blocks] partial sums of E^bc, then [B] E^bc
    int pen_blocks;
    size_t bytes;      // total workspace
};

// Validates `spec` and fills `plan` for batch B (B may be 1 for size queries).
dmcr_status make_plan(const dmcr_spec *spec, int B, Plan *plan);

// ---- kernel timing (dmcr_profile_start / dmcr_profile_stop) ---------------
bool prof_on();
// A start/stop event pair for one launch of `name` (both null if none is left).
void prof_pair(const char *name, double bytes, hipEvent_t *start, hipEvent_t *stop);

// Launch `kernel` on `st`.  While timing is on, the launch carries a start/stop
// event pair that the runtime stamps from the dispatch itself (the kernel's own
// begin and end, as a kernel trace reports them), so the timing adds no stream
// commands between kernels.
template <typename Kern, typename... Args>
hipError_t launch(const char *name, double bytes, Kern kernel, dim3 grid, dim3 block, size_t lds,
                  hipStream_t st, Args... args)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (prof_on()) prof_pair(name, bytes, &a, &b);
    if (a && b)
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, st, a, b, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
    return hipGetLastError();
}

// ---- launchers (all asynchronous on `st`) ---------------------------------
struct Ws {
    char *base;
    template <class T> T *at(size_t off) const { return reinterpret_cast<T *>(base + off); }
};

hipError_t launch_restrict(const Plan &p, int l, const float *fine, float *coarse, hipStream_t st);
// levels l+1 and l+2 from level l in one pass (bitwise as two launch_restrict)
hipError_t launch_restrict2(const Plan &p, int l, const float *fine, float *mid, float *coarse, hipStream_t st);
hipError_t launch_prolong_add(const Plan &p, int l, const float *coarse_grad, float *fine_grad,
                              hipStream_t st);
// fine (level l) = nearest-neighbour upsampling of coarse (level l + 1)
hipError_t launch_upsample(const Plan &p, int l, const float *coarse, float *fine, hipStream_t st);
hipError_t run_pyramid_levels(const Plan &p, const float *phi, const Ws &ws, hipStream_t st);

// x_free (optional) is recorded on st once the partial spectrum X of the level
// has been consumed, so that a recompute of X on another stream may start.
hipError_t fft_forward_level(const Plan &p, int l, const float *phi, float *S, const Ws &ws,
                             hipStream_t st, hipEvent_t x_free = nullptr);
// fused = false keeps the two-pass transforms of 3-D levels (for a spectrum
// computed while other kernels of the same step run on other streams).  With
// msum, the first pass also writes float64 partial sums of every field
// (fft_mean_parts per field, in field order).
hipError_t fft_spectrum_level(const Plan &p, int l, const float *phi, const Ws &ws, hipStream_t st,
                              bool fused = true, double *msum = nullptr);
// partial sums per field that the first forward pass of level l writes
int64_t fft_mean_parts(const Plan &p, int l);
// Without have_spectrum the spectrum is recomputed: on st_spec after x_free when
// st_spec is given (overlapping the cotangent transforms on st), else on st.
// With St, G is the descriptor S and the cotangent 2 w_l^2 (S - St) / Z of the
// loss is formed while loading (bitwise as the error kernel forms it), so the
// adjoint need not wait for the error kernel.
// With coarse (only where fft_fused_prolong holds), the last inverse pass also
// adds the prolongation of the next coarser level's total gradient, 2^-d times
// each voxel's parent, after st waits for coarse_ready (if given).
hipError_t fft_adjoint_level(const Plan &p, int l, const float *phi, const float *G, float *grad,
                             bool have_spectrum, const Ws &ws, hipStream_t st, hipStream_t st_spec = nullptr,
                             hipEvent_t x_free = nullptr, hipEvent_t spec_done = nullptr,
                             const double *St = nullptr, const float *coarse = nullptr,
                             hipEvent_t coarse_ready = nullptr);
// Whether level l's adjoint ends in an inverse pass that can add the
// prolongation: the fused plane transform, or the contiguous-axis inverse with
// rows of at least 4 (FFT path).
bool fft_fused_prolong(const Plan &p, int l);

// 3-D levels with square planes of side 32..256: the contiguous axis and axis 1
// transformed in one pass (fft_plane.hip).  Forward: real field [B][C][n0][n][n]
// -> half spectra X [B][C][n0][n][hp]; inverse: X -> real field (unnormalised).
bool plane_supported(const Plan &p, int l);
// waves per plane workgroup (one partial sum of the mean each)
int plane_waves(const Plan &p, int l);
// With msum, also float64 sums of every wave's share of each plane, at
// msum[plane * plane_waves + wave].
hipError_t plane_forward(const Plan &p, int l, const float *phi, float2 *X, hipStream_t st, double *msum = nullptr);
// With coarse, the inverse also adds 1/8 of the coarser level's gradient at each
// voxel's parent (the multigrid prolongation; needs an even n0).
hipError_t plane_inverse(const Plan &p, int l, const float2 *X, float *grad, hipStream_t st,
                         const float *coarse = nullptr);

hipError_t direct_forward_level(const Plan &p, int l, const float *phi, float *S, const Ws &ws,
                                hipStream_t st);
// With St, G is the descriptor S and the cotangent 2 w_l^2 (S - St) / Z is formed
// by the kernel-building pass (bitwise as the error kernel forms it), so the
// level's adjoint need not wait for the error kernel.
hipError_t direct_adjoint_level(const Plan &p, int l, const float *phi, const float *G, float *grad,
                                const Ws &ws, hipStream_t st, const double *St = nullptr);

hipError_t launch_build_kernels(const Plan &p, int l, const float *G, float *KB0, hipStream_t st,
                                const double *St = nullptr);

// Appendix A map of the soft-threshold descriptor (DMCR_DESC_STILDE), in place
// on S [B][K], and its transpose from G_in to G_out (may be the same array).
hipError_t launch_stilde(const Plan &p, float *S, hipStream_t st);
hipError_t launch_stilde_adjoint(const Plan &p, const float *G_in, float *G_out, hipStream_t st);

// Three-point blocks of level l: forward into S, adjoint added into grad (the
// level gradient written by the two-point adjoint).  The Appendix A map of the
// three-point blocks (STILDE) in place on S, and its transpose in place on G
// (run before launch_stilde_adjoint; it adds into the two-point cotangents).
// choose the contraction kernels of level l's three-point blocks (fills s3mf,
// s3VB, s3VBa, s3bf, s3ba, s3Kp, s3Mp, s3chunks; none depends on the batch, so a
// field's result does not either); false if unsupported
bool s3_configure(Plan &p, int l);
hipError_t s3_forward_level(const Plan &p, int l, const float *phi, float *S, const Ws &ws, hipStream_t st);
// With St, G is the descriptor S and the three-point cotangents 2 w_l^2 (S - St) / Z
// are formed while reading it (bitwise as the error kernel forms them).
hipError_t s3_adjoint_level(const Plan &p, int l, const float *phi, const float *G, float *grad, const Ws &ws,
                            hipStream_t st, const double *St = nullptr);
hipError_t launch_s3_map(const Plan &p, float *S, hipStream_t st);
hipError_t launch_s3_map_adjoint(const Plan &p, float *G, hipStream_t st);

// E and the cotangent G from S.  G is ready on st; with st_final (and the
// event parts_done) the final sum into E runs on st_final instead, off the
// path of the adjoint, and the caller joins st_final.
hipError_t launch_error(const Plan &p, const float *S, const double *St, double *E, float *G,
                        const Ws &ws, hipStream_t st, hipStream_t st_final = nullptr,
                        hipEvent_t parts_done = nullptr);

// forward, error and adjoint with one plan (dmcr_loss_grad, the solvers).  With
// lanes = false everything runs on st (no internal streams or events are created).
dmcr_status loss_grad_internal(const Plan &p, const float *phi, const double *St, double *E, float *grad,
                               const Ws &w, hipStream_t st, bool lanes = true);

// true if the DIRECT path can run this level (halo tile fits in LDS)
bool direct_supported(const Plan &p, int l, int tile_out[3]);

}  // namespace dmcr
