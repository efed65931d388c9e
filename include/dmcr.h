/*
 * dmcr.h -- C ABI of libdmcr, the MI355X (gfx950) library for the
 * differentiable multigrid two-point-correlation descriptor of
 * Seibert, Ambati, Rassloff, Kaestner, "Reconstructing random heterogeneous
 * media through differentiable optimization" (arXiv 2103.09686).
 *
 * The problem it serves (Sec. 3.1, eq. dMCR-Min_Prob): find a real-valued
 * field M~ minimising L(M~) = E(M~) + lambda E^bc(M~), where the descriptor
 * D~ = f~_C(M~) (eq. fctilde) is the multigrid concatenation of eq. (mg) of
 * two-point correlations, and the box 0 <= M~ <= 1 is the bound of Sec. 3.1.
 *
 * Conventions shared by every call
 * --------------------------------
 * Fields.  A batch of B independent problems.  Each holds C explicit soft
 *   phase indicators phi_c (C = number of phases - 1; the matrix phase is
 *   1 - sum_c phi_c and carries no extra information, Sec. 3.2.1).  Layout
 *   float32 [B][C][n0][n1] (2-D) or [B][C][n0][n1][n2] (3-D), last axis
 *   contiguous, every axis a power of two.
 * Levels.  Level 0 is the caller's field; level l+1 is the 2^d mean pool of
 *   level l (Sec. 3.3: a coarse pixel summarises 2^{d} finer ones).
 * Correlations.  For level l, pair (i, j) and displacement r:
 *       S_ij^(l)(r) = (1/N_l) sum_x phi_i^(l)(x) phi_j^(l)((x + r) mod n_l)
 *   (Sec. 3.2.1-3.2.2 with the periodic shift of eq. convdef; for soft
 *   fields this is the Appendix A corrected descriptor with the identity
 *   threshold used in Sec. 5.1).  spec.descriptor selects the paper's
 *   soft-threshold form instead (see DMCR_DESC_*), and spec.s3_max_disp adds
 *   three-point blocks (eq. s3).  Auto pairs (i == j) use the half box H_P
 *   (r = 0 or first non-zero component > 0; point symmetry, Appendix B),
 *   cross pairs the full box [-P, P]^d.
 * Descriptor order.  Level-major (finest first), then pair in the order of
 *   spec.pairs, then r lexicographic with axis 0 slowest.  Values are
 *   unweighted; the level weights w_l (eq. mg) enter only the error.
 * Error.  E = (1/Z) sum_l w_l^2 sum_{pairs} sum_r (S - S_target)^2,
 *   Z = sum_l w_l^2 K_l (K_l = entries of level l): the squared form of the
 *   descriptor distance of Sec. 3.1, normalised per entry.
 * Memory.  The caller owns every buffer.  Pointers marked "device" must be
 *   device memory of the current HIP device; the library never allocates on
 *   these calls: scratch comes from the caller's workspace `ws` of at least
 *   dmcr_workspace_size() bytes (256-byte aligned).  Fields, gradients,
 *   pyramid levels and float64 buffers must be 8-byte aligned (fields move as
 *   float pairs); a 16-byte aligned field lets the pyramid restrict two levels
 *   per pass.  A misaligned pointer returns DMCR_EINVAL.
 * Streams.  Every call except the reconstruction and solver-slot calls is
 *   asynchronous on `stream` and returns before the work finishes; device
 *   faults surface on a later call or synchronisation.  Calls that share a
 *   workspace must not overlap.
 * Errors.  Arguments are validated before any launch; on error nothing is
 *   launched and a negative dmcr_status is returned.  No call aborts.
 */
#ifndef DMCR_H
#define DMCR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DMCR_OK = 0,
    DMCR_EINVAL = -1,        /* bad argument: null pointer, bad shape, P too large, ... */
    DMCR_ENOMEM = -2,        /* workspace smaller than dmcr_workspace_size()            */
    DMCR_EUNSUPPORTED = -3,  /* valid problem this library does not handle (e.g. DIRECT
                                path with a halo tile larger than LDS)                  */
    DMCR_EDEVICE = -4,       /* a HIP call failed (launch or runtime error)             */
    DMCR_ENONFINITE = -5,    /* reconstruct: loss or gradient became NaN / Inf          */
    DMCR_NOT_CONVERGED = 1,  /* reconstruct: iteration budget spent before tolerance    */
    DMCR_RUNNING = 2         /* solver slot: still iterating                            */
} dmcr_status;

enum { DMCR_MAX_LEVELS = 8, DMCR_MAX_CHANNELS = 4, DMCR_MAX_PAIRS = 10 };

/* Evaluation path.  AUTO picks per level; FFT uses the convolution theorem
 * (Stockham transforms in LDS); DIRECT sums shifted products over an LDS
 * tile with a halo of P (the paper's own convolve-and-reduce, Sec. 3.2.3). */
enum { DMCR_PATH_AUTO = 0, DMCR_PATH_FFT = 1, DMCR_PATH_DIRECT = 2 };

/* spec.descriptor: which two-point statistic each (level, pair) block holds.
 *   S2     the product form (1/N) sum_x phi_i(x) phi_j(x + r): the Appendix A
 *          corrected descriptor of the identity threshold (Sec. 5.1).
 *   SBAR   the paper's soft-threshold descriptor (Sec. 3.2.4, eq. softthreshold,
 *          and eq. s3 with r_a = r_b): (1/N) sum_x f((phi_i(x) + phi_j(x + r)) / 2)^2
 *          with the logistic f(u) = c1 / (1 + exp(-alpha (u + c2))) + c3 fixed by
 *          f(0) = 0, f(1) = 1, f''(0.75) = 0.  The r = 0 mask of an auto pair
 *          gives f(phi_i(x)), the same expression.
 *   STILDE SBAR mapped back by Appendix A, eq. (s2rfroms2rbar): with F = f(1/2)^2,
 *          (SBAR_ij(r) - F (SBAR_ii(0) + SBAR_jj(0))) / (1 - 2F); equals S2 on
 *          binary fields.  Every channel of a listed pair needs its auto pair.
 * SBAR and STILDE are evaluated on the DIRECT path only (AUTO selects it; FFT
 * returns DMCR_EUNSUPPORTED): the soft threshold is not a product, so the
 * convolution theorem does not apply. */
enum { DMCR_DESC_S2 = 0, DMCR_DESC_SBAR = 1, DMCR_DESC_STILDE = 2 };

/* Three-point correlations (Sec. 3.2.2, eq. s3), spec.s3_max_disp = P3 > 0.  Each
 * level l appends, after its two-point blocks, one block per channel c holding
 *     S3_c(r_a, r_b) = (1/N) sum_x e_a(x) e_b(x)
 * for every unordered pair r_a <= r_b (index order) of the M = (2 P3_l + 1)^d
 * vectors of [-P3_l, P3_l]^d in lexicographic order (axis 0 slowest), P3_l =
 * min(P3, P_l); the block has M (M + 1) / 2 entries, r_a-major.  The realisation
 * product e_a e_b is phi(x) phi(x + r_a) phi(x + r_b) with DMCR_DESC_S2 (the exact
 * three-point probability on binary fields) and f(u_a) f(u_b), u_c = (phi(x) +
 * phi(x + r_c)) / 2, with the soft-threshold descriptors; STILDE maps it back
 * by Appendix A, eq. (s3rfroms3rbar), from the mapped two-point values, which
 * needs 2 P3_l <= P_l and the auto pair of every channel.  Evaluated by
 * dedicated kernels on every path; larger vector sets (M > 361: 2-D P3 > 9,
 * 3-D P3 > 3) return DMCR_EUNSUPPORTED. */

/* spec.flags */
enum {
    DMCR_FLAG_RECOMPUTE = 1,    /* dmcr_loss_grad recomputes the forward spectra in the
                                   adjoint instead of keeping them between the two halves */
    DMCR_FLAG_FUSED_PLANES = 2  /* FFT path, 3-D levels with 256 x 256 planes: transform the
                                   contiguous axis and axis 1 in one pass (one plane per
                                   workgroup) instead of two.  Levels with square planes of
                                   side 32..128 always do.  Fewer HBM bytes; at 256 the fused
                                   pass holds a whole compute unit per plane and cannot
                                   overlap its loads with its stores */
};

typedef struct {
    int32_t ndim;                          /* 2 or 3                                  */
    int32_t shape[3];                      /* finest level, powers of two, >= 2       */
    int32_t n_channels;                    /* C, 1..DMCR_MAX_CHANNELS                 */
    int32_t n_levels;                      /* 1..DMCR_MAX_LEVELS; every axis must be
                                              divisible by 2^(n_levels-1).  0 selects
                                              the level rule of Appendix B (P = 31:
                                              1, 2, 3 levels at 64, 128, 256):
                                              L = max(1, 1 + round(log2(min_axis /
                                              (2 (P + 1))))), P = max_disp[0] on every
                                              level, default weights               */
    int32_t max_disp[DMCR_MAX_LEVELS];     /* P_l >= 0; clipped to min_axis(n_l)/2 - 1
                                              (a longer displacement aliases)          */
    double  level_weight[DMCR_MAX_LEVELS]; /* w_l (eq. mg), > 0; 0 selects the default
                                              2^{d l / 2} (level 0 finest), the square
                                              root of the voxels a coarse voxel
                                              summarises (2^{l-1} of eq. mg's footnote,
                                              1-based, in 2-D)                          */
    int32_t n_pairs;                       /* 0 = all pairs i <= j in lexicographic order */
    int32_t pairs[2 * 16];                 /* (i, j) with i <= j, used if n_pairs > 0 */
    int32_t path;                          /* DMCR_PATH_*                             */
    int32_t flags;                         /* DMCR_FLAG_*                             */
    int32_t descriptor;                    /* DMCR_DESC_*                             */
    int32_t s3_max_disp;                   /* P3 > 0 appends a three-point block per
                                              channel and level (see below); 0 = none */
    double  alpha;                         /* soft-threshold slope (SBAR, STILDE);
                                              0 selects the paper's 10                */
} dmcr_spec;

/* Box handling for dmcr_reconstruct (Sec. 3.1). */
enum { DMCR_BOUNDS_NONE = 0, DMCR_BOUNDS_PROJECT = 1, DMCR_BOUNDS_PENALTY = 2 };
typedef struct {
    double lo, hi;   /* the box, normally [0, 1]                                          */
    int32_t mode;    /* PROJECT: iterates are clipped to [lo, hi] and the search direction
                        is restricted to free variables; PENALTY: L = E + lambda E^bc with
                        E^bc as printed in Sec. 3.1 and lambda = kappa E held constant in
                        the gradient and in the Armijo test of a line search started at
                        that point (see dmcr_penalised_loss_grad)                          */
    double kappa;
} dmcr_bounds;

/* Optimizer of dmcr_reconstruct and the solver slots.  LBFGS: batched projected
 * L-BFGS with backtracking.  ADAM: the paper's optimizer (Appendix B; Kingma &
 * Ba, Alg. 1) with projection onto the box after each step; one evaluation per
 * iteration, no line search. */
enum { DMCR_OPT_LBFGS = 0, DMCR_OPT_ADAM = 1 };

typedef struct {
    int32_t m;          /* L-BFGS history length (1..32; ignored by ADAM)      */
    int32_t max_iter;   /* iteration budget                                    */
    int32_t max_ls;     /* evaluations per line search (ignored by ADAM)       */
    double  tol_derr;   /* stop when E <= tol_derr                             */
    double  c1;         /* Armijo sufficient-decrease constant, (0, 1); the
                           backtracking search halves the step until it holds  */
    int32_t method;     /* DMCR_OPT_*                                          */
    double  lr;         /* ADAM: step size (the paper: 1e-3), > 0              */
    double  beta1;      /* ADAM: first-moment decay (0.9), in [0, 1)           */
    double  beta2;      /* ADAM: second-moment decay (0.999), in [0, 1)        */
    double  eps;        /* ADAM: denominator guard (1e-7), > 0                 */
} dmcr_opt;

typedef struct {
    double  final_E;     /* E of the returned field                           */
    double  final_derr;  /* same quantity (the weighted mean squared error)   */
    int32_t iters;       /* iterations taken                                  */
    int32_t evals;       /* loss/gradient evaluations                         */
    int32_t why;         /* dmcr_status for this batch element                */
} dmcr_result;

/* Number of multigrid levels L of the spec (spec->n_levels, or the level rule
 * when it is 0); < 0: dmcr_status. */
int32_t dmcr_level_count(const dmcr_spec *spec);

/* Number of descriptor entries K (all levels and pairs); < 0: dmcr_status. */
int64_t dmcr_descriptor_size(const dmcr_spec *spec);

/* Offsets of every block in descriptor order: per level, each pair's two-point
 * block, then (s3_max_disp > 0) each channel's three-point block; writes
 * L * (n_pairs + (s3_max_disp > 0 ? n_channels : 0)) + 1 values (L from
 * dmcr_level_count; the last one is K) to host array `offsets`. */
dmcr_status dmcr_descriptor_offsets(const dmcr_spec *spec, int64_t *offsets);

/* Workspace bytes needed by every call below for this spec and batch size. */
dmcr_status dmcr_workspace_size(const dmcr_spec *spec, int32_t batch, size_t *bytes);

/* Multigrid pyramid (Sec. 3.3): writes levels 1..L-1 of phi, each the 2^d
 * mean pool of the previous, concatenated level after level into `levels`
 * (device, float32, sum_l B*C*N_l values). */
dmcr_status dmcr_pyramid(const dmcr_spec *spec, int32_t batch, const float *phi, float *levels,
                         hipStream_t stream);

/* Forward descriptor (Sec. 3.2-3.3): phi (device [B][C][n...]) -> S (device
 * float32 [B][K]). */
dmcr_status dmcr_descriptor_forward(const dmcr_spec *spec, int32_t batch, const float *phi,
                                    float *S, void *ws, size_t ws_bytes, hipStream_t stream);

/* Adjoint (the gradient the method back-propagates through every level at
 * once, Sec. 3.3): grad = d/dphi sum_{b,k} dS[b][k] S[b][k], overwriting
 * grad (device [B][C][n...]).  The spectra of phi are recomputed. */
dmcr_status dmcr_descriptor_adjoint(const dmcr_spec *spec, int32_t batch, const float *phi,
                                    const float *dS, float *grad, void *ws, size_t ws_bytes,
                                    hipStream_t stream);

/* Error and cotangent: E[b] (device float64) and G = dE/dS (device
 * float32 [B][K]) from S (device float32 [B][K]) and S_target (device
 * float64 [B][K]); the sum is taken in float64 in a fixed order. */
dmcr_status dmcr_error_cotangent(const dmcr_spec *spec, int32_t batch, const float *S,
                                 const double *S_target, double *E, float *G, void *ws,
                                 size_t ws_bytes, hipStream_t stream);

/* One optimiser evaluation: forward, error, adjoint.  E (device float64 [B]),
 * grad (device float32 [B][C][n...], overwritten). */
dmcr_status dmcr_loss_grad(const dmcr_spec *spec, int32_t batch, const float *phi,
                           const double *S_target, double *E, float *grad, void *ws,
                           size_t ws_bytes, hipStream_t stream);

/* dmcr_loss_grad without a workspace argument, for callers that cannot allocate
 * (code under stream capture, serving loops that must not call an allocator):
 * the scratch memory is a 64 MiB device array inside the library, one copy per
 * device, held until the process ends.  A spec and batch whose workspace
 * (dmcr_workspace_size) exceeds 64 MiB returns DMCR_ENOMEM before any launch.
 * Everything runs on `stream` (no internal streams); nothing is allocated.  All
 * calls on one device share that array: calls that overlap in time on one
 * device (concurrent streams or host threads) race and must not be issued.
 * Arguments and results as dmcr_loss_grad. */
dmcr_status dmcr_loss_grad_noalloc(const dmcr_spec *spec, int32_t batch, const float *phi, const double *S_target,
                                   double *E, float *grad, hipStream_t stream);

/* The loss of the relaxed problem (Sec. 3.1, eq. L_func_dMCR) and its gradient:
 * with bounds->mode == DMCR_BOUNDS_PENALTY, L[b] = E[b] + lambda E^bc[b], where
 * E^bc = sum_c sum_x [ (phi - hi) H(phi - hi) / N + (lo - phi) H(lo - phi) / N ]^2
 * (the printed penalty with the box [lo, hi], H(0) = 0, N voxels per channel)
 * and lambda = kappa E[b], held constant in the gradient
 * grad = dE/dphi + lambda dE^bc/dphi; with any other mode L = E and grad = dE/dphi.
 * L, E: device float64 [B]; grad: device float32 [B][C][n...], overwritten;
 * workspace: dmcr_workspace_size().  Asynchronous on `stream`. */
dmcr_status dmcr_penalised_loss_grad(const dmcr_spec *spec, int32_t batch, const float *phi, const double *S_target,
                                     const dmcr_bounds *bounds, double *L, double *E, float *grad, void *ws,
                                     size_t ws_bytes, hipStream_t stream);

/* Workspace bytes for dmcr_reconstruct (includes dmcr_workspace_size). */
dmcr_status dmcr_reconstruct_workspace_size(const dmcr_spec *spec, int32_t batch,
                                            const dmcr_opt *opt, size_t *bytes);

/* Reconstruction (Sec. 3, Fig. 1 loop): minimise E (+ penalty) over phi with
 * L-BFGS or Adam (opt->method), starting from phi_inout (device [B][C][n...], overwritten with the
 * result).  S_target: device float64 [B][K].  results: host array of B.
 * Blocking: synchronises `stream` before returning.  Returns DMCR_OK if every
 * element reached tol_derr, DMCR_NOT_CONVERGED if some did not, or an error. */
dmcr_status dmcr_reconstruct(const dmcr_spec *spec, int32_t batch, const double *S_target,
                             const dmcr_bounds *bounds, const dmcr_opt *opt, float *phi_inout,
                             dmcr_result *results, void *ws, size_t ws_bytes, hipStream_t stream);

/* Sequential coarse-to-fine reconstruction: the level-by-level multigrid
 * practice that Sec. 3.3 contrasts with its simultaneous scheme, for comparison.
 * The start field is mean-pooled to the coarsest level; each level l, coarsest
 * first, is reconstructed alone (the single-level spec of level l, weight 1)
 * against the level-l slice of the multigrid target S_target ([B][K], device),
 * with up to opt->max_iter iterations; its result, upsampled by nearest
 * neighbour, starts level l - 1.  phi_inout receives the finest result.
 * results[b]: final_E is the multigrid error of the result against the whole
 * target, iters and evals are summed over the levels (evals includes the final
 * evaluation); why is DMCR_OK if final_E <= tol_derr.  Workspace:
 * dmcr_reconstruct_c2f_workspace_size.  Blocking, like dmcr_reconstruct. */
dmcr_status dmcr_reconstruct_c2f_workspace_size(const dmcr_spec *spec, int32_t batch, const dmcr_opt *opt,
                                                size_t *bytes);
dmcr_status dmcr_reconstruct_coarse_to_fine(const dmcr_spec *spec, int32_t batch, const double *S_target,
                                            const dmcr_bounds *bounds, const dmcr_opt *opt, float *phi_inout,
                                            dmcr_result *results, void *ws, size_t ws_bytes, hipStream_t stream);

/* Kernel timing (diagnostics).  dmcr_profile_start() clears the table and
 * makes every later launch of the evaluation kernels carry a HIP event pair
 * that the runtime stamps with the dispatch's own begin and end
 * (hipExtLaunchKernel), with the launch's algorithmic bytes (inputs read once
 * plus outputs written once).  dmcr_profile_stop() synchronises on the
 * recorded events, writes at most `max` per-kernel totals to `out` (host) and
 * returns the number of distinct kernels (or a negative dmcr_status).
 * Process-global and not thread-safe; do not record while a stream is being
 * captured. */
typedef struct {
    char name[48];
    int32_t launches;
    double total_ms;
    double bytes;     /* algorithmic bytes summed over the launches */
} dmcr_kernel_stat;

dmcr_status dmcr_profile_start(void);
int32_t dmcr_profile_stop(dmcr_kernel_stat *out, int32_t max);

/* Continuous batching.  A solver batch of B slots shares one spec, one field
 * buffer phi [B][C][n...], one target buffer S_target [B][K] (float64, device)
 * and one workspace of dmcr_reconstruct_workspace_size() bytes; the per-slot
 * scalars live in a host array of B dmcr_slot and the shared history ring in a
 * dmcr_ring (initialise head = opt->m - 1, count = 0).  Slots are independent:
 * each slot's iterates are bitwise the same whatever the other slots hold.
 *   dmcr_solver_start   (re)starts the listed slots from their current phi:
 *                       projection, one evaluation, empty history (Adam: zero
 *                       moments); sets active = 1 and status = RUNNING (or OK /
 *                       ENONFINITE).
 *   dmcr_solver_iterate runs up to `iterations` L-BFGS or Adam iterations of
 *                       every slot with active = 1 and status = RUNNING; a slot
 *                       stops with OK (E <= tol_derr), NOT_CONVERGED (iters >=
 *                       max_iter or a stalled line search) or ENONFINITE.
 * Both synchronise `stream` before returning.  The caller clears `active` of a
 * slot it retires and may then start a new request in it. */
typedef struct {
    double  f;        /* current loss (E plus penalty)        */
    double  E;        /* current descriptor error             */
    int32_t hist;     /* pairs in this slot's history         */
    int32_t iters;    /* iterations since start               */
    int32_t evals;    /* evaluations since start              */
    int32_t status;   /* dmcr_status: RUNNING, OK, NOT_CONVERGED, ENONFINITE */
    int32_t active;   /* 1 while the slot holds a request     */
    int32_t reserved;
} dmcr_slot;

typedef struct {
    int32_t head, count;   /* newest history position, positions in use */
} dmcr_ring;

dmcr_status dmcr_solver_start(const dmcr_spec *spec, int32_t batch, const int32_t *which, int32_t nwhich,
                              const double *S_target, const dmcr_bounds *bounds, const dmcr_opt *opt, float *phi,
                              dmcr_slot *slots, void *ws, size_t ws_bytes, hipStream_t stream);
dmcr_status dmcr_solver_iterate(const dmcr_spec *spec, int32_t batch, const double *S_target,
                                const dmcr_bounds *bounds, const dmcr_opt *opt, float *phi, dmcr_slot *slots,
                                dmcr_ring *ring, int32_t iterations, void *ws, size_t ws_bytes, hipStream_t stream);

/* Static description of a status code. */
const char *dmcr_status_string(dmcr_status status);

#ifdef __cplusplus
}
#endif
#endif /* DMCR_H */
