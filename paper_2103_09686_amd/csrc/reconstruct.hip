// Reconstruction driver (the loop of Fig. 1 / eq. M-update, Sec. 3): batched
// limited-memory BFGS on the relaxed problem of eq. (dMCR-Min_Prob).
//
// Every vector operation runs on the device in float32 with float64 dot
// products (fixed-order, deterministic reductions).  Each batch element keeps
// its own history (rho = 0 marks an empty or rejected slot), step length and
// status; elements advance in lockstep because one loss/gradient evaluation
// covers the whole batch.  The host reads back only the per-element scalars
// each decision needs (loss, penalty, directional derivatives).
//
// Direction: the compact representation of the L-BFGS inverse Hessian (Byrd,
// Nocedal & Schnabel, Math. Prog. 63, 1994, Thm. 2.2) with H0 = gamma I, gamma =
// s'y / y'y of the newest accepted pair:
//   H g = gamma g + S p - gamma Y q,  q = R^-1 S'g,  p = R^-T ((D + gamma Y'Y) q - gamma Y'g),
// R the upper triangle of S'Y over the element's valid pairs in age order, D its
// diagonal.  It equals the two-loop recursion (Nocedal & Wright, Alg. 7.4) in
// exact arithmetic, but needs only one pass of dot products over the history,
// an O(m^2) float64 solve per element and one pass of linear combination,
// instead of 2m dependent dot/update passes.  S'Y and Y'Y are kept per element
// and extended by one row and column per accepted pair.  Box handling
// (Sec. 3.1): PROJECT clips trial points to [lo, hi] and zeroes direction
// components that push an active bound outward; PENALTY adds lambda E^bc with
// E^bc as printed in Sec. 3.1 and lambda = kappa * E held constant in the
// gradient and in the Armijo test of a search started at that point.  Step:
// backtracking (halving) along the projected path with the Armijo test
// f(x_t) <= f(x) + c1 g'(x_t - x), first trial 1 (1/|g| without history); a
// pair (s, y) enters the history only if s'y > eps y'y.  A failed
// line search clears that element's history; a failure that started from
// steepest descent stops the element.
//
// Adam (the paper's optimizer, Appendix B; Kingma & Ba, Alg. 1): per element the
// biased moments m, v (in the first history slot), bias corrections 1 - beta^t
// at the element's own step count t, the step lr m_hat / (sqrt(v_hat) + eps),
// then projection onto the box; one evaluation per iteration.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "dmcr_internal.h"

namespace dmcr {

namespace {

constexpr int kV = 256;

size_t align_up_bytes(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

unsigned vblocks(int64_t n) { return (unsigned)std::min<int64_t>((n + kV - 1) / kV, 2048); }

// Deterministic sum of one element's block partials: thread t adds partials
// t, t + kV, ... in order, then a fixed tree.  One block per element.
__device__ __forceinline__ double block_sum(const double *p, int cnt, int64_t stride, double *red)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < cnt; i += kV) s += p[i * stride];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kV / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    return red[0];
}

// out[b] = sum of part[b][0 .. nblk)   (grid: one block of kV threads per element)
__global__ __launch_bounds__(kV) void k_sum_parts(const double *part, int nblk, double *out, int B)
{
    __shared__ double red[kV];
    const int64_t b = blockIdx.x;
    const double s = block_sum(part + b * nblk, nblk, 1, red);
    if (threadIdx.x == 0) out[b] = s;
}

__global__ void k_fill(double *p, double v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// History dot products, one pass over the ring slots j < cnt in use, per element
// b, fused with the acceptance of a trial point: with acc and acc[b], first
//   s = xt - x, y = gt - g into ring slot `slot`, x = xt, g = gt
// (the accepted step and its pair), then
//   [j] = S_j.g, [m + j] = Y_j.g, [2m] = g.g
// and, for an accepted element (its new pair in slot `slot`),
//   [2m + 1 + j] = s_j.y, [3m + 1 + j] = y_j.y, [4m + 1 + j] = s.y_j.
// acc null: the dots of the current g only.  One pass reads every vector once
// (up to kHistJ ring slots; a longer ring takes more passes).  Fixed order
// throughout: strided element loop, wave shuffles, waves in order; the sums are
// bitwise those of a separate accept followed by a dots pass.
constexpr int kMaxDots = 5 * 32 + 1;
constexpr int kHistJ = 10;  // ring slots per pass (5 kHistJ + 1 float64 accumulators)

__device__ __forceinline__ int hist_count(int cnt, bool pair) { return 2 * cnt + 1 + (pair ? 3 * cnt : 0); }

__device__ __forceinline__ int hist_out(int k, int cnt, int m)
{
    if (k < cnt) return k;
    if (k < 2 * cnt) return m + (k - cnt);
    if (k == 2 * cnt) return 2 * m;
    k -= 2 * cnt + 1;
    if (k < cnt) return 2 * m + 1 + k;
    if (k < 2 * cnt) return 3 * m + 1 + (k - cnt);
    return 4 * m + 1 + (k - 2 * cnt);
}

__global__ __launch_bounds__(kV) void k_accept_dots(const int *acc, float *x, const float *xt, float *g,
                                                    const float *gt, float *Sb, float *Yb, int slot, int cnt, int m,
                                                    int B, int64_t n, double *part, int nblk)
{
    constexpr int NA = 5 * kHistJ + 1;
    __shared__ double red[kV / 64][NA];
    const int64_t b = blockIdx.y;
    const int64_t stride = (int64_t)B * n;
    const bool pair = acc != nullptr && acc[b] != 0;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    double *pb = part + ((int64_t)b * nblk + blockIdx.x) * kMaxDots;
    float *Sn = Sb + (int64_t)(slot < 0 ? 0 : slot) * stride, *Yn = Yb + (int64_t)(slot < 0 ? 0 : slot) * stride;
    for (int c0 = 0; c0 < cnt || c0 == 0; c0 += kHistJ) {
        const int cj = min(kHistJ, cnt - c0);
        double a[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) a[k] = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < n; i += (int64_t)nblk * kV) {
            const int64_t e = b * n + i;
            // every slot of the pass is loaded before the accepted step, so that all
            // loads are in flight together (an index past the ring reads slot 0 and
            // its sums are never stored); the new pair comes from registers, so the
            // slot it replaces is not read (a condition uniform over the block)
            float svf[kHistJ], yvf[kHistJ];
#pragma unroll
            for (int jj = 0; jj < kHistJ; ++jj) {
                const int j = c0 + jj < cnt ? c0 + jj : 0;
                svf[jj] = yvf[jj] = 0.f;
                if (!(pair && c0 + jj == slot)) {
                    svf[jj] = Sb[(int64_t)j * stride + e];
                    yvf[jj] = Yb[(int64_t)j * stride + e];
                }
            }
            float gf, sf = 0.f, yf = 0.f;
            if (pair && c0 == 0) {          // the accepted step, once
                const float xo = x[e], xn = xt[e], go = g[e], gn = gt[e];
                sf = xn - xo;
                yf = gn - go;
                Sn[e] = sf;
                Yn[e] = yf;
                x[e] = xn;
                g[e] = gn;
                gf = gn;
            } else {
                gf = g[e];
                if (pair) {                  // later passes: the pair as the first one wrote it
                    sf = Sn[e];
                    yf = Yn[e];
                }
            }
            const double gv = gf, yn = yf, sn = sf;
            if (c0 == 0) a[NA - 1] += gv * gv;
            if (pair) {
#pragma unroll
                for (int jj = 0; jj < kHistJ; ++jj) {
                    const bool nw = c0 + jj == slot;
                    const double sv = nw ? sf : svf[jj], yv = nw ? yf : yvf[jj];
                    a[5 * jj + 0] += sv * gv;
                    a[5 * jj + 1] += yv * gv;
                    a[5 * jj + 2] += sv * yn;
                    a[5 * jj + 3] += yv * yn;
                    a[5 * jj + 4] += sn * yv;
                }
            } else {
#pragma unroll
                for (int jj = 0; jj < kHistJ; ++jj) {
                    const double sv = svf[jj], yv = yvf[jj];
                    a[5 * jj + 0] += sv * gv;
                    a[5 * jj + 1] += yv * gv;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NA; ++k)
            for (int off = 32; off > 0; off >>= 1) a[k] += __shfl_down(a[k], off);
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < NA; ++k) red[wave][k] = a[k];
        __syncthreads();
        if (threadIdx.x < NA) {
            const int k = threadIdx.x;
            double sum = 0.0;
            for (int w = 0; w < kV / 64; ++w) sum += red[w][k];
            if (k == NA - 1) {
                if (c0 == 0) pb[2 * m] = sum;
            } else {
                const int jj = k / 5, r = k % 5, j = c0 + jj;
                if (jj < cj && (r < 2 || pair)) {
                    const int o = r == 0 ? j : r == 1 ? m + j : r == 2 ? 2 * m + 1 + j : r == 3 ? 3 * m + 1 + j
                                                                                          : 4 * m + 1 + j;
                    pb[o] = sum;
                }
            }
        }
        __syncthreads();
    }
}

// dots[b kMaxDots + o] = sum over the blocks' partials (grid: element b x dot k)
__global__ __launch_bounds__(kV) void k_hist_sum(const double *part, int nblk, int cnt, int m, double *dots)
{
    __shared__ double red[kV];
    const int64_t b = blockIdx.x;
    const int o = hist_out(blockIdx.y, cnt, m);
    const double s = block_sum(part + b * nblk * kMaxDots + o, nblk, kMaxDots, red);
    if (threadIdx.x == 0) dots[b * kMaxDots + o] = s;
}

// Compact-representation coefficients of element b (one thread each):
// dots[j] = S_j.g, dots[m + j] = Y_j.g (ring slot j), dots[2m] = g.g;
// SY[b][i][j] = s_i.y_j, YY[b][i][j] = y_i.y_j.  Valid pairs (rho != 0) in age
// order from the oldest; H g = cg g + sum_j cS_j S_j + cY_j Y_j.
__global__ void k_lbfgs_coef(const double *dots, const double *rho, const double *gamma, const double *SY,
                             const double *YY, int head, int count, int m, int B, double *cS, double *cY, double *cg,
                             double *gg)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double *db = dots + (int64_t)b * kMaxDots;
    const double *sy = SY + (int64_t)b * m * m, *yy = YY + (int64_t)b * m * m;
    int idx[32];
    int k = 0;
    for (int t = count - 1; t >= 0; --t) {
        const int i = (head - t + m) % m;
        if (rho[(int64_t)i * B + b] != 0.0) idx[k++] = i;
    }
    const double gam = gamma[b];
    double q[32], pc[32];
    for (int u = k - 1; u >= 0; --u) {            // R q = S'g (back substitution)
        double acc = db[idx[u]];
        for (int v = u + 1; v < k; ++v) acc -= sy[idx[u] * m + idx[v]] * q[v];
        q[u] = acc / sy[idx[u] * m + idx[u]];
    }
    for (int u = 0; u < k; ++u) {                 // R' p = D q + gamma Y'Y q - gamma Y'g
        double acc = sy[idx[u] * m + idx[u]] * q[u] - gam * db[m + idx[u]];
        for (int v = 0; v < k; ++v) acc += gam * yy[idx[u] * m + idx[v]] * q[v];
        for (int v = 0; v < u; ++v) acc -= sy[idx[v] * m + idx[u]] * pc[v];
        pc[u] = acc / sy[idx[u] * m + idx[u]];
    }
    for (int i = 0; i < m; ++i) {
        cS[(int64_t)b * m + i] = 0.0;
        cY[(int64_t)b * m + i] = 0.0;
    }
    for (int u = 0; u < k; ++u) {
        cS[(int64_t)b * m + idx[u]] = pc[u];
        cY[(int64_t)b * m + idx[u]] = -gam * q[u];
    }
    cg[b] = gam;
    gg[b] = db[2 * m];
}

// d = -(cg g + sum_j cS_j S_j + cY_j Y_j) over the ring slots in use, oldest
// first (so that an element's sum runs in the same order wherever its pairs sit
// in the shared ring), with projection: components that push an active bound
// outward are zeroed.  A zero coefficient skips its history vector (which may
// hold nothing valid).  part = block partials of g . d.
__global__ __launch_bounds__(kV) void k_combine_dir(const float *x, const float *g, float *d, const float *Sb,
                                                    const float *Yb, const double *cS, const double *cY,
                                                    const double *cg, int m, int head, int count, int B, int64_t n,
                                                    int project, float lo, float hi, double *part, int nblk)
{
    __shared__ float cs[32], cy[32];
    __shared__ double red[kV];
    const int64_t b = blockIdx.y;
    if (threadIdx.x < count) {
        cs[threadIdx.x] = (float)cS[b * m + threadIdx.x];
        cy[threadIdx.x] = (float)cY[b * m + threadIdx.x];
    }
    __syncthreads();
    const float c0 = (float)cg[b];
    const int64_t stride = (int64_t)B * n;
    constexpr int kChunk = 10;  // history slots whose loads are issued together
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < n; i += (int64_t)nblk * kV) {
        const int64_t j = b * n + i;
        const float gv = g[j];
        float h = c0 * gv;
        for (int t0 = count - 1; t0 >= 0; t0 -= kChunk) {
            float sv[kChunk], yv[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {   // unconditional loads (t < 0 reads the newest slot, unused)
                const int t = t0 - u;
                const int k = (head - (t < 0 ? 0 : t) + m) % m;
                sv[u] = Sb[k * stride + j];
                yv[u] = Yb[k * stride + j];
            }
            // oldest first; a slot with a zero coefficient is skipped (it may hold nothing valid)
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const int t = t0 - u;
                if (t >= 0) {
                    const int k = (head - t + m) % m;
                    if (cs[k] != 0.f) h += cs[k] * sv[u];
                    if (cy[k] != 0.f) h += cy[k] * yv[u];
                }
            }
        }
        const float xv = x[j];
        float dv = -h;
        if (project && ((xv <= lo && dv < 0.f) || (xv >= hi && dv > 0.f))) dv = 0.f;
        d[j] = dv;
        acc += (double)gv * (double)dv;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kV / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[b * nblk + blockIdx.x] = red[0];
}

// New pair in ring slot `slot` (written by k_accept_dots for accepted elements):
// dots[2m + 1 + j] = s_j.y_new, [3m + 1 + j] = y_j.y_new, [4m + 1 + j] = s_new.y_j (j < count).
// rho = 1/s'y if accepted and s'y > eps y'y, else 0; gamma follows; the slot's
// row and column of S'Y and Y'Y are refreshed.
__global__ void k_pair_update(const double *dots, const int *acc, int slot, int count, int m, int B, double *rho,
                              double *gamma, double *SY, double *YY)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    if (!acc[b]) {
        rho[(int64_t)slot * B + b] = 0.0;
        return;
    }
    const double *db = dots + (int64_t)b * kMaxDots;
    const double *sjy = db + 2 * m + 1, *yjy = db + 3 * m + 1, *sny = db + 4 * m + 1;
    const double sy = sny[slot], yy = yjy[slot];
    const bool ok = sy > 2.220446049250313e-16 * yy && yy > 0.0;
    rho[(int64_t)slot * B + b] = ok ? 1.0 / sy : 0.0;
    if (ok) gamma[b] = sy / yy;
    double *syb = SY + (int64_t)b * m * m, *yyb = YY + (int64_t)b * m * m;
    for (int j = 0; j < count; ++j) {
        syb[slot * m + j] = sny[j];
        syb[j * m + slot] = sjy[j];
        yyb[slot * m + j] = yjy[j];
        yyb[j * m + slot] = yjy[j];
    }
}

// clear the history of one element
__global__ void k_reset_one(double *rho, double *gamma, int m, int B, int b)
{
    if (threadIdx.x == 0) {
        for (int i = 0; i < m; ++i) rho[i * B + b] = 0.0;
        gamma[b] = 1.0;
    }
}

// clear the history of flagged elements
__global__ void k_reset(const int *flag, double *rho, double *gamma, int m, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B || !flag[b]) return;
    for (int i = 0; i < m; ++i) rho[i * B + b] = 0.0;
    gamma[b] = 1.0;
}

// After the direction, per element: one whose d is not a descent direction
// (g.d >= 0) falls back to projected steepest descent (flag) with a cleared
// history; the first trial step is 1/|g| without history, else 1.
__global__ void k_dir_check(const double *gd, const double *gg, const int *active, const int *hist, int *flag,
                            double *rho, double *gamma, double *step, int m, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int f = active[b] && !(gd[b] < 0.0);
    flag[b] = f;
    if (f) {
        for (int i = 0; i < m; ++i) rho[(int64_t)i * B + b] = 0.0;
        gamma[b] = 1.0;
    }
    const double gn = sqrt(gg[b]);
    step[b] = ((f || hist[b] == 0) && gn > 0.0) ? 1.0 / gn : 1.0;
}

// dst[k] = src[idx[k]] (rows of len elements), k < gridDim.y
template <class T>
__global__ __launch_bounds__(kV) void k_gather(const int *idx, const T *src, T *dst, int64_t len)
{
    const int64_t k = blockIdx.y, b = idx[k];
    for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < len; i += (int64_t)gridDim.x * kV)
        dst[k * len + i] = src[b * len + i];
}

// dst[idx[k]] = src[k]
template <class T>
__global__ __launch_bounds__(kV) void k_scatter(const int *idx, const T *src, T *dst, int64_t len)
{
    const int64_t k = blockIdx.y, b = idx[k];
    for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < len; i += (int64_t)gridDim.x * kV)
        dst[b * len + i] = src[k * len + i];
}

// Trial point xt = x + alpha d (clipped with projection) of the active elements,
// and block partials of g . (xt - x), the Armijo test's directional term, in
// float64 over a strided element loop and a fixed tree (zero for inactive
// elements).
__global__ __launch_bounds__(kV) void k_trial_dot(const float *x, const float *d, const float *g, const double *alpha,
                                                  const int *active, float *xt, int64_t n, int project, float lo,
                                                  float hi, double *part, int nblk)
{
    __shared__ double red[kV];
    const int64_t b = blockIdx.y;
    double acc = 0.0;
    if (active[b]) {
        const float a = (float)alpha[b];
        for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < n; i += (int64_t)nblk * kV) {
            const int64_t j = b * n + i;
            const float xv = x[j];
            float v = xv + a * d[j];
            if (project) v = fminf(fmaxf(v, lo), hi);
            xt[j] = v;
            acc += (double)g[j] * ((double)v - (double)xv);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kV / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[b * nblk + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kV) void k_clip(float *x, int64_t total, float lo, float hi)
{
    for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < total; i += (int64_t)gridDim.x * kV)
        x[i] = fminf(fmaxf(x[i], lo), hi);
}

// d = -d; with projection, components that push an active bound outward are zeroed
__global__ __launch_bounds__(kV) void k_finish_dir(const float *x, float *d, int64_t n, int project, float lo, float hi)
{
    const int64_t b = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < n; i += (int64_t)gridDim.x * kV) {
        const float xv = x[b * n + i];
        float dv = -d[b * n + i];
        if (project && ((xv <= lo && dv < 0.f) || (xv >= hi && dv > 0.f))) dv = 0.f;
        d[b * n + i] = dv;
    }
}

// flagged elements: d = -g (projected as above)
__global__ __launch_bounds__(kV) void k_steepest(const int *flag, const float *x, const float *g, float *d, int64_t n,
                                                 int project, float lo, float hi)
{
    const int64_t b = blockIdx.y;
    if (!flag[b]) return;
    for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < n; i += (int64_t)gridDim.x * kV) {
        const float xv = x[b * n + i];
        float dv = -g[b * n + i];
        if (project && ((xv <= lo && dv < 0.f) || (xv >= hi && dv > 0.f))) dv = 0.f;
        d[b * n + i] = dv;
    }
}

// Adam step of running elements (status RUNNING, step t = iters + 1):
// m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// x -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), clipped to [lo, hi] with projection
__global__ __launch_bounds__(kV) void k_adam(float *x, const float *g, float *mm, float *vv, const int *status,
                                             const int *iters, int64_t n, float lr, double beta1, double beta2,
                                             float eps, int project, float lo, float hi)
{
    const int64_t b = blockIdx.y;
    if (status[b] != DMCR_RUNNING) return;
    const int t = iters[b] + 1;
    const float b1 = (float)beta1, b2 = (float)beta2;
    const float ic1 = (float)(1.0 / (1.0 - pow(beta1, (double)t)));
    const float ic2 = (float)(1.0 / (1.0 - pow(beta2, (double)t)));
    for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < n; i += (int64_t)gridDim.x * kV) {
        const int64_t j = b * n + i;
        const float gi = g[j];
        const float m = b1 * mm[j] + (1.f - b1) * gi;
        const float v = b2 * vv[j] + (1.f - b2) * gi * gi;
        mm[j] = m;
        vv[j] = v;
        float xv = x[j] - lr * (m * ic1) / (sqrtf(v * ic2) + eps);
        if (project) xv = fminf(fmaxf(xv, lo), hi);
        x[j] = xv;
    }
}

// after an Adam step's evaluation: count it and decide each running element's status
__global__ void k_adam_check(const double *E, const double *Ebc, double kappa, int penalty, double tol, int max_iter,
                             double *f, int *iters, int *evals, int *status, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B || status[b] != DMCR_RUNNING) return;
    ++iters[b];
    ++evals[b];
    const double fb = E[b] + (penalty ? kappa * E[b] * Ebc[b] : 0.0);
    f[b] = fb;
    if (!isfinite(fb))
        status[b] = DMCR_ENONFINITE;
    else if (E[b] <= tol)
        status[b] = DMCR_OK;
    else if (iters[b] >= max_iter)
        status[b] = DMCR_NOT_CONVERGED;
}

__global__ __launch_bounds__(kV) void k_zero(float *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < n; i += (int64_t)gridDim.x * kV) p[i] = 0.f;
}

// E^bc = sum_i t_i^2 with t = (x-hi)H(x-hi)/N + (lo-x)H(lo-x)/N, H(0) = 0 (per channel N)
__global__ __launch_bounds__(kV) void k_pen_part(const float *x, int64_t n, double invN, float lo, float hi,
                                                 double *part, int nblk)
{
    __shared__ double red[kV];
    const int64_t b = blockIdx.y;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < n; i += (int64_t)nblk * kV) {
        const double v = x[b * n + i];
        const double t = (v > hi ? (v - hi) : 0.0) * invN + (v < lo ? (lo - v) : 0.0) * invN;
        acc += t * t;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kV / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[b * nblk + blockIdx.x] = red[0];
}

// g += kappa E dE^bc/dx,  dE^bc/dx = 2 t (H(x-hi) - H(lo-x)) / N
__global__ __launch_bounds__(kV) void k_pen_grad(const float *x, float *g, const double *E, double kappa, int64_t n,
                                                 double invN, float lo, float hi)
{
    const int64_t b = blockIdx.y;
    const double lam = kappa * E[b];
    for (int64_t i = (int64_t)blockIdx.x * kV + threadIdx.x; i < n; i += (int64_t)gridDim.x * kV) {
        const double v = x[b * n + i];
        const double t = (v > hi ? (v - hi) : 0.0) * invN + (v < lo ? (lo - v) : 0.0) * invN;
        const double dt = (v > hi ? invN : 0.0) - (v < lo ? invN : 0.0);
        g[b * n + i] += (float)(lam * 2.0 * t * dt);
    }
}

// L[b] = E[b] + kappa E[b] E^bc[b]   (Ebc null: L = E)
__global__ void k_pen_loss(const double *E, const double *Ebc, double kappa, double *L, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) L[b] = E[b] + (Ebc ? kappa * E[b] * Ebc[b] : 0.0);
}

struct RLayout {
    size_t xt, g, gt, d, s, y;
    size_t part, dot1, dot2, rho, gamma, E, Et, Ebc, als, active, acc, flag;
    size_t SY, YY, cS, cY, cg, mdots, mpart;   // L-BFGS compact representation
    size_t sl_f, sl_iters, sl_evals, sl_status;   // Adam: per-slot state kept on the device
    size_t histd;                                 // L-BFGS: each element's history length
    size_t pk_idx, pk_x, pk_g, pk_St, pk_E, pk_Ebc;   // packed evaluation of B' < B elements
    int nblk;
    size_t bytes;
};

RLayout r_layout(const Plan &p, const dmcr_opt &o)
{
    RLayout r{};
    const int64_t n = (int64_t)p.C * p.lv[0].N;
    const size_t Bn = (size_t)p.B * n;
    size_t top = align_up_bytes(p.bytes);
    auto take = [&](size_t bytes) {
        const size_t at = top;
        top = align_up_bytes(top + bytes);
        return at;
    };
    const size_t B8 = (size_t)p.B * 8;
    r.xt = take(Bn * 4);
    r.g = take(Bn * 4);
    r.gt = take(Bn * 4);
    r.d = take(Bn * 4);
    const int hist = (o.method == DMCR_OPT_ADAM) ? 1 : o.m;   // Adam keeps m, v in slot 0
    r.s = take((size_t)hist * Bn * 4);
    r.y = take((size_t)hist * Bn * 4);
    // enough blocks per element to keep the loads of a large field in flight
    r.nblk = (int)std::max<int64_t>(1, std::min<int64_t>(2048, (n + 4 * kV - 1) / (4 * kV)));
    r.part = take((size_t)p.B * r.nblk * 8);
    r.dot1 = take(B8);
    r.dot2 = take(B8);
    r.rho = take((size_t)o.m * B8);
    r.gamma = take(B8);
    r.SY = take((size_t)o.m * o.m * B8);
    r.YY = take((size_t)o.m * o.m * B8);
    r.cS = take((size_t)o.m * B8);
    r.cY = take((size_t)o.m * B8);
    r.cg = take(B8);
    r.mdots = take((size_t)kMaxDots * B8);
    r.mpart = take((size_t)r.nblk * kMaxDots * B8);
    r.E = take(B8);
    r.Et = take(B8);
    r.Ebc = take(B8);
    r.als = take(B8);
    r.active = take((size_t)p.B * 4);
    r.acc = take((size_t)p.B * 4);
    r.flag = take((size_t)p.B * 4);
    r.sl_f = take(B8);
    r.sl_iters = take((size_t)p.B * 4);
    r.sl_evals = take((size_t)p.B * 4);
    r.sl_status = take((size_t)p.B * 4);
    r.histd = take((size_t)p.B * 4);
    const size_t Bp = (size_t)std::max(0, p.B - 1);   // at most B - 1 elements are packed
    r.pk_idx = take((size_t)p.B * 4);
    r.pk_x = take(Bp * n * 4);
    r.pk_g = take(Bp * n * 4);
    r.pk_St = take(Bp * p.K * 8);
    r.pk_E = take(B8);
    r.pk_Ebc = take(B8);
    r.bytes = top;
    return r;
}

bool opt_ok(const dmcr_opt *o)
{
    if (!o || o->max_iter < 0 || !std::isfinite(o->tol_derr)) return false;
    if (o->method == DMCR_OPT_ADAM)
        return o->lr > 0 && std::isfinite(o->lr) && o->beta1 >= 0 && o->beta1 < 1 && o->beta2 >= 0 &&
               o->beta2 < 1 && o->eps > 0 && std::isfinite(o->eps) && o->m >= 1 && o->m <= 32;
    return o->method == DMCR_OPT_LBFGS && o->m >= 1 && o->m <= 32 && o->max_ls >= 1 && o->c1 > 0 && o->c1 < 1;
}

#define RT(expr)                                               \
    do {                                                       \
        if ((expr) != hipSuccess) return DMCR_EDEVICE;         \
    } while (0)
#define RS(expr)                                               \
    do {                                                       \
        dmcr_status _s = (expr);                               \
        if (_s != DMCR_OK) return _s;                          \
    } while (0)

// Pinned host staging for the line search's device-to-host reads (trial errors,
// directional dots, first steps, history flags): with a pinned destination the
// copies are asynchronous and the search's one synchronisation covers them all,
// where pageable ones are staged one at a time.  One area per host thread, grown
// as needed and kept until the process ends.  A solver call that succeeds ends
// synchronised; one that returned an error may have left copies into the area in
// flight, so growing it first waits for the device.
struct PinnedStage {
    void *p = nullptr;
    size_t bytes = 0;
};
thread_local PinnedStage tl_pin;

hipError_t pinned_stage(size_t bytes, void **out)
{
    if (tl_pin.bytes < bytes) {
        if (tl_pin.p) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return e;
            e = hipHostFree(tl_pin.p);
            tl_pin.p = nullptr;
            tl_pin.bytes = 0;
            if (e != hipSuccess) return e;
        }
        hipError_t e = hipHostMalloc(&tl_pin.p, bytes, hipHostMallocPortable);
        if (e != hipSuccess) {
            tl_pin.p = nullptr;
            return e;
        }
        tl_pin.bytes = bytes;
    }
    *out = tl_pin.p;
    return hipSuccess;
}

struct Solver {
    const Plan &p;
    const dmcr_bounds &bd;
    const dmcr_opt &o;
    const double *St;
    RLayout r;
    Ws w;
    hipStream_t st;
    int B, m;
    int64_t n;
    dim3 vg, sg;
    bool project, penalty;
    float lo, hi;
    double invN;

    template <class T> T *at(size_t off) const { return w.at<T>(off); }
    float *S(int i) const { return at<float>(r.s) + (int64_t)i * B * n; }
    float *Y(int i) const { return at<float>(r.y) + (int64_t)i * B * n; }

    // history dot products of the ring slots 0 .. cnt - 1 against g and, with
    // acc (accepted elements; their step enters ring slot `slot` and x, g move to
    // xt, gt in the same pass), against the new pair; summed into mdots
    hipError_t hist_dots(float *x, const float *xt, float *g, const float *gt, const int *acc, int cnt,
                         int slot) const
    {
        hipLaunchKernelGGL(k_accept_dots, dim3(r.nblk, B), dim3(kV), 0, st, acc, x, xt, g, gt, S(0), Y(0), slot,
                           cnt, m, B, n, at<double>(r.mpart), r.nblk);
        const int nout = 2 * cnt + 1 + (slot >= 0 ? 3 * cnt : 0);
        hipLaunchKernelGGL(k_hist_sum, dim3(B, nout), dim3(kV), 0, st, at<double>(r.mpart), r.nblk, cnt, m,
                           at<double>(r.mdots));
        return hipGetLastError();
    }

    dmcr_status evaluate(const float *pt, double *Ed, float *grad) const
    {
        RS(loss_grad_internal(p, pt, St, Ed, grad, w, st));
        if (penalty) {
            hipLaunchKernelGGL(k_pen_part, dim3(r.nblk, B), dim3(kV), 0, st, pt, n, invN, lo, hi, at<double>(r.part),
                               r.nblk);
            hipLaunchKernelGGL(k_sum_parts, dim3(B), dim3(kV), 0, st, at<double>(r.part), r.nblk, at<double>(r.Ebc), B);
            hipLaunchKernelGGL(k_pen_grad, vg, dim3(kV), 0, st, pt, grad, Ed, bd.kappa, n, invN, lo, hi);
            RT(hipGetLastError());
        }
        return DMCR_OK;
    }

    dmcr_status fetch(const double *src, std::vector<double> &dst) const
    {
        RT(hipMemcpyAsync(dst.data(), src, B * sizeof(double), hipMemcpyDeviceToHost, st));
        return DMCR_OK;
    }

    dmcr_status fetch_int(const int *src, std::vector<int> &dst) const
    {
        RT(hipMemcpyAsync(dst.data(), src, B * sizeof(int), hipMemcpyDeviceToHost, st));
        return DMCR_OK;
    }

    dmcr_status put(int *dst, const std::vector<int> &src) const
    {
        RT(hipMemcpyAsync(dst, src.data(), B * sizeof(int), hipMemcpyHostToDevice, st));
        return DMCR_OK;
    }

    dmcr_status put(double *dst, const std::vector<double> &src) const
    {
        RT(hipMemcpyAsync(dst, src.data(), B * sizeof(double), hipMemcpyHostToDevice, st));
        return DMCR_OK;
    }

    dmcr_spec spec1;  // the spec, for batch-1 plans of single-slot evaluations
    Ws w1;            // same workspace base (a batch-1 plan fits inside the batch-B one)

    // Loss and gradient of the trial points of the elements with act[b] only,
    // when they are fewer than B: gathered into a batch of B' = count elements
    // (the evaluation of an element does not depend on the batch it is in),
    // evaluated, and scattered back into Ed, grad (and the penalty's E^bc).
    mutable std::vector<int> pk_host;   // the packed indices, alive until the next call

    dmcr_status evaluate_packed(const std::vector<int> &act, const float *pt, double *Ed, float *grad) const
    {
        std::vector<int> &idx = pk_host;
        idx.clear();
        for (int b = 0; b < B; ++b)
            if (act[b]) idx.push_back(b);
        const int bp = (int)idx.size();
        idx.resize(B, 0);
        int *idxd = at<int>(r.pk_idx);
        float *px = at<float>(r.pk_x), *pg = at<float>(r.pk_g);
        double *pS = at<double>(r.pk_St), *pE = at<double>(r.pk_E), *pEbc = at<double>(r.pk_Ebc);
        RS(put(idxd, idx));
        const dim3 gv(vblocks(n), bp), gk(vblocks(p.K), bp), g1(1, bp);
        hipLaunchKernelGGL(k_gather<float>, gv, dim3(kV), 0, st, idxd, pt, px, n);
        hipLaunchKernelGGL(k_gather<double>, gk, dim3(kV), 0, st, idxd, St, pS, p.K);
        RT(hipGetLastError());
        Plan pb;
        dmcr_spec sb = spec1;
        RS(make_plan(&sb, bp, &pb));
        RS(loss_grad_internal(pb, px, pS, pE, pg, w1, st));
        if (penalty) {
            hipLaunchKernelGGL(k_pen_part, dim3(r.nblk, bp), dim3(kV), 0, st, px, n, invN, lo, hi, at<double>(r.part),
                               r.nblk);
            hipLaunchKernelGGL(k_sum_parts, dim3(bp), dim3(kV), 0, st, at<double>(r.part), r.nblk, pEbc, bp);
            hipLaunchKernelGGL(k_pen_grad, gv, dim3(kV), 0, st, px, pg, pE, bd.kappa, n, invN, lo, hi);
            hipLaunchKernelGGL(k_scatter<double>, g1, dim3(kV), 0, st, idxd, pEbc, at<double>(r.Ebc), (int64_t)1);
        }
        hipLaunchKernelGGL(k_scatter<float>, gv, dim3(kV), 0, st, idxd, pg, grad, n);
        hipLaunchKernelGGL(k_scatter<double>, g1, dim3(kV), 0, st, idxd, pE, Ed, (int64_t)1);
        RT(hipGetLastError());
        return DMCR_OK;
    }

    dmcr_status start(float *x, const int *which, int nwhich, dmcr_slot *slots);
    dmcr_status iterate(float *x, dmcr_slot *slots, dmcr_ring *ring, int iterations);
    dmcr_status iterate_adam(float *x, dmcr_slot *slots, int iterations);
};

// (Re)start the listed slots: clip (PROJECT), evaluate loss and gradient of each
// slot on its own (batch-1 evaluations, bitwise identical to the batched ones),
// clear its history.
dmcr_status Solver::start(float *x, const int *which, int nwhich, dmcr_slot *slots)
{
    float *g = at<float>(r.g);
    double *rho = at<double>(r.rho), *gamma = at<double>(r.gamma);
    double *Ed = at<double>(r.E), *Ebcd = at<double>(r.Ebc);
    Plan p1;
    dmcr_spec one = spec1;
    RS(make_plan(&one, 1, &p1));
    // every started slot's E (and E^bc) lands in the pinned area; one synchronisation
    // after the last evaluation (they share the batch-1 workspace in stream order)
    void *pin = nullptr;
    RT(pinned_stage((size_t)2 * B * sizeof(double), &pin));
    double *pE = static_cast<double *>(pin), *pEbc = pE + B;
    for (int w = 0; w < nwhich; ++w) {
        const int b = which[w];
        float *xb = x + (int64_t)b * n;
        float *gb = g + (int64_t)b * n;
        if (project)
            hipLaunchKernelGGL(k_clip, dim3(vblocks(n)), dim3(kV), 0, st, xb, n, lo, hi);
        RS(loss_grad_internal(p1, xb, St + (int64_t)b * p.K, Ed + b, gb, w1, st));
        if (penalty) {
            hipLaunchKernelGGL(k_pen_part, dim3(r.nblk, 1), dim3(kV), 0, st, xb, n, invN, lo, hi, at<double>(r.part),
                               r.nblk);
            hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kV), 0, st, at<double>(r.part), r.nblk, Ebcd + b, 1);
            hipLaunchKernelGGL(k_pen_grad, dim3(vblocks(n), 1), dim3(kV), 0, st, xb, gb, Ed + b, bd.kappa, n, invN, lo,
                               hi);
        }
        hipLaunchKernelGGL(k_reset_one, dim3(1), dim3(64), 0, st, rho, gamma, m, B, b);
        if (o.method == DMCR_OPT_ADAM) {   // fresh moments
            hipLaunchKernelGGL(k_zero, dim3(vblocks(n)), dim3(kV), 0, st, S(0) + (int64_t)b * n, n);
            hipLaunchKernelGGL(k_zero, dim3(vblocks(n)), dim3(kV), 0, st, Y(0) + (int64_t)b * n, n);
        }
        RT(hipGetLastError());
        RT(hipMemcpyAsync(pE + b, Ed + b, 8, hipMemcpyDeviceToHost, st));
        if (penalty) RT(hipMemcpyAsync(pEbc + b, Ebcd + b, 8, hipMemcpyDeviceToHost, st));
    }
    RT(hipStreamSynchronize(st));
    for (int w = 0; w < nwhich; ++w) {
        const int b = which[w];
        const double E = pE[b], Ebc = penalty ? pEbc[b] : 0.0;
        dmcr_slot &sl = slots[b];
        sl.E = E;
        sl.f = E + (penalty ? bd.kappa * E * Ebc : 0.0);
        sl.hist = 0;
        sl.iters = 0;
        sl.evals = 1;
        sl.active = 1;
        sl.status = DMCR_RUNNING;
        if (!std::isfinite(sl.f))
            sl.status = DMCR_ENONFINITE;
        else if (sl.E <= o.tol_derr)
            sl.status = DMCR_OK;
    }
    return DMCR_OK;
}

// Up to `iterations` Adam steps of every running slot.  The per-slot counters
// and the stopping decisions live on the device, so steps are queued without a
// host round trip; the host checks every kCheck steps whether any slot still runs.
dmcr_status Solver::iterate_adam(float *x, dmcr_slot *slots, int iterations)
{
    constexpr int kCheck = 16;
    float *g = at<float>(r.g);
    double *Ed = at<double>(r.E), *Ebcd = at<double>(r.Ebc), *fd = at<double>(r.sl_f);
    int *itd = at<int>(r.sl_iters), *evd = at<int>(r.sl_evals), *std_ = at<int>(r.sl_status);
    std::vector<int> hit(B), hev(B), hst(B);
    std::vector<double> hf(B), hE(B);
    for (int b = 0; b < B; ++b) {
        hit[b] = slots[b].iters;
        hev[b] = slots[b].evals;
        hst[b] = (slots[b].active && slots[b].status == DMCR_RUNNING) ? DMCR_RUNNING : DMCR_OK;
        hf[b] = slots[b].f;
    }
    RS(put(itd, hit));
    RS(put(evd, hev));
    RS(put(std_, hst));
    RS(put(fd, hf));
    for (int it = 0; it < iterations; ++it) {
        if (it % kCheck == 0) {
            RS(fetch_int(std_, hst));
            RT(hipStreamSynchronize(st));
            bool any = false;
            for (int b = 0; b < B; ++b) any |= hst[b] == DMCR_RUNNING;
            if (!any) break;
        }
        hipLaunchKernelGGL(k_adam, vg, dim3(kV), 0, st, x, g, S(0), Y(0), std_, itd, n, (float)o.lr, o.beta1, o.beta2,
                           (float)o.eps, (int)project, lo, hi);
        RT(hipGetLastError());
        RS(evaluate(x, Ed, g));
        hipLaunchKernelGGL(k_adam_check, sg, dim3(64), 0, st, Ed, Ebcd, bd.kappa, (int)penalty, o.tol_derr,
                           o.max_iter, fd, itd, evd, std_, B);
        RT(hipGetLastError());
    }
    RS(fetch_int(itd, hit));
    RS(fetch_int(evd, hev));
    RS(fetch_int(std_, hst));
    RS(fetch(fd, hf));
    RS(fetch(Ed, hE));
    RT(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b) {
        if (!(slots[b].active && slots[b].status == DMCR_RUNNING)) continue;
        dmcr_slot &sl = slots[b];
        if (hit[b] == sl.iters) continue;   // took no step
        sl.iters = hit[b];
        sl.evals = hev[b];
        sl.status = hst[b];
        sl.f = hf[b];
        sl.E = hE[b];
    }
    return DMCR_OK;
}

// Up to `iterations` L-BFGS iterations of every running slot.
dmcr_status Solver::iterate(float *x, dmcr_slot *slots, dmcr_ring *ring, int iterations)
{
    if (o.method == DMCR_OPT_ADAM) return iterate_adam(x, slots, iterations);
    float *xt = at<float>(r.xt), *g = at<float>(r.g), *gt = at<float>(r.gt), *d = at<float>(r.d);
    double *rho = at<double>(r.rho), *gamma = at<double>(r.gamma);
    double *dot1 = at<double>(r.dot1), *dot2 = at<double>(r.dot2);
    double *Etd = at<double>(r.Et), *Ebcd = at<double>(r.Ebc), *als = at<double>(r.als);
    double *SY = at<double>(r.SY), *YY = at<double>(r.YY), *cS = at<double>(r.cS), *cY = at<double>(r.cY);
    double *cg = at<double>(r.cg), *mdots = at<double>(r.mdots);
    int *active = at<int>(r.active), *accd = at<int>(r.acc), *flagd = at<int>(r.flag);

    std::vector<double> hE(B), hEbc(B, 0.0), hd(B), step(B);
    std::vector<int> act(B), acc(B), flag(B), hist(B);
    int *histd = at<int>(r.histd);
    void *pin = nullptr;   // pinned landing area of the line search's reads: E, Ebc, dot, step, flag
    RT(pinned_stage((size_t)B * (4 * sizeof(double) + sizeof(int)), &pin));
    double *pE = static_cast<double *>(pin), *pEbc = pE + B, *pd = pE + 2 * B, *pstep = pE + 3 * B;
    int *pflag = reinterpret_cast<int *>(pE + 4 * B);
    const size_t db = (size_t)B * sizeof(double), ib = (size_t)B * sizeof(int);
    auto running = [&](int b) { return slots[b].active && slots[b].status == DMCR_RUNNING; };
    int head = ring->head, count = ring->count;
    bool gdots = false;   // mdots holds S'g, Y'g, g'g of the current g and history

    for (int it = 0; it < iterations; ++it) {
        bool any = false;
        for (int b = 0; b < B; ++b) any |= running(b);
        if (!any) break;

        for (int b = 0; b < B; ++b) {
            act[b] = running(b);
            acc[b] = 0;
            hist[b] = slots[b].hist;
        }
        RS(put(active, act));
        RS(put(histd, hist));

        // ---- direction d = -H g (compact representation), then projection ----
        if (!gdots) RT(hist_dots(x, nullptr, g, nullptr, nullptr, count, -1));
        hipLaunchKernelGGL(k_lbfgs_coef, sg, dim3(64), 0, st, mdots, rho, gamma, SY, YY, head, count, m, B, cS, cY,
                           cg, dot2);
        hipLaunchKernelGGL(k_combine_dir, dim3(r.nblk, B), dim3(kV), 0, st, x, g, d, S(0), Y(0), cS, cY, cg, m, head,
                           count, B, n, (int)project, lo, hi, at<double>(r.part), r.nblk);
        hipLaunchKernelGGL(k_sum_parts, dim3(B), dim3(kV), 0, st, at<double>(r.part), r.nblk, dot1, B);
        // not a descent direction: (projected) steepest descent; first step, on the device
        hipLaunchKernelGGL(k_dir_check, sg, dim3(64), 0, st, dot1, dot2, active, histd, flagd, rho, gamma, als, m, B);
        hipLaunchKernelGGL(k_steepest, vg, dim3(kV), 0, st, flagd, x, g, d, n, (int)project, lo, hi);
        RT(hipGetLastError());

        // ---- backtracking line search along the projected path ----
        for (int ls = 0; ls < o.max_ls; ++ls) {
            bool anyact = false;
            for (int b = 0; b < B; ++b) anyact |= act[b] != 0;
            if (!anyact) break;
            if (ls > 0) {
                RS(put(active, act));
                RS(put(als, step));
            }
            hipLaunchKernelGGL(k_trial_dot, dim3(r.nblk, B), dim3(kV), 0, st, x, d, g, als, active, xt, n,
                               (int)project, lo, hi, at<double>(r.part), r.nblk);
            hipLaunchKernelGGL(k_sum_parts, dim3(B), dim3(kV), 0, st, at<double>(r.part), r.nblk, dot1, B);
            int nact = 0;
            for (int b = 0; b < B; ++b) nact += act[b] != 0;
            if (nact < B)
                RS(evaluate_packed(act, xt, Etd, gt));   // backtracking elements only, or a partly idle batch
            else
                RS(evaluate(xt, Etd, gt));
            RT(hipMemcpyAsync(pE, Etd, db, hipMemcpyDeviceToHost, st));
            if (penalty) RT(hipMemcpyAsync(pEbc, Ebcd, db, hipMemcpyDeviceToHost, st));
            RT(hipMemcpyAsync(pd, dot1, db, hipMemcpyDeviceToHost, st));
            if (ls == 0) {
                RT(hipMemcpyAsync(pstep, als, db, hipMemcpyDeviceToHost, st));
                RT(hipMemcpyAsync(pflag, flagd, ib, hipMemcpyDeviceToHost, st));
            }
            RT(hipStreamSynchronize(st));
            std::copy(pE, pE + B, hE.begin());
            if (penalty) std::copy(pEbc, pEbc + B, hEbc.begin());
            std::copy(pd, pd + B, hd.begin());
            if (ls == 0) {
                std::copy(pstep, pstep + B, step.begin());
                std::copy(pflag, pflag + B, flag.begin());
            }
            if (ls == 0)
                for (int b = 0; b < B; ++b)
                    if (flag[b]) slots[b].hist = 0;   // the device cleared its history
            for (int b = 0; b < B; ++b) {
                if (!act[b]) continue;
                ++slots[b].evals;
                // the Armijo test holds lambda = kappa E of the search's start point,
                // as the gradient there does; an accepted point's f takes its own lambda
                const double ft = hE[b] + (penalty ? bd.kappa * slots[b].E * hEbc[b] : 0.0);
                if (std::isfinite(ft) && hd[b] < 0.0 && ft <= slots[b].f + o.c1 * hd[b]) {
                    act[b] = 0;
                    acc[b] = 1;
                    slots[b].f = hE[b] + (penalty ? bd.kappa * hE[b] * hEbc[b] : 0.0);
                    slots[b].E = hE[b];
                } else {
                    step[b] *= 0.5;
                }
            }
        }

        // ---- update the field, gradient and history of accepted elements ----
        const int slot = (head + 1) % m;
        RS(put(accd, acc));
        const int cnew = std::min(count + 1, m);   // ring slots in use: 0 .. cnew - 1
        // accepted steps enter slot `slot`; the new pair's dots and the next direction's
        RT(hist_dots(x, xt, g, gt, accd, cnew, slot));
        gdots = true;
        hipLaunchKernelGGL(k_pair_update, sg, dim3(64), 0, st, mdots, accd, slot, cnew, m, B, rho, gamma, SY, YY);
        RT(hipGetLastError());
        head = slot;
        count = cnew;
        bool any_fail = false;
        for (int b = 0; b < B; ++b) {
            flag[b] = 0;
            if (!running(b)) continue;
            dmcr_slot &sl = slots[b];
            ++sl.iters;
            if (acc[b]) {
                sl.hist = std::min(sl.hist + 1, m);
                if (sl.E <= o.tol_derr) sl.status = DMCR_OK;
            } else {
                flag[b] = 1;  // clear the history of a failed line search
                any_fail = true;
                if (sl.hist == 0) sl.status = DMCR_NOT_CONVERGED;  // no progress even from steepest descent
                sl.hist = 0;
            }
            if (sl.status == DMCR_RUNNING && sl.iters >= o.max_iter) sl.status = DMCR_NOT_CONVERGED;
        }
        if (any_fail) {
            RS(put(flagd, flag));
            hipLaunchKernelGGL(k_reset, sg, dim3(64), 0, st, flagd, rho, gamma, m, B);
            RT(hipGetLastError());
        }
    }
    ring->head = head;
    ring->count = count;
    RT(hipStreamSynchronize(st));
    return DMCR_OK;
}

}  // namespace
}  // namespace dmcr

using namespace dmcr;

namespace {

dmcr_status make_solver(const dmcr_spec *spec, int32_t batch, const double *S_target, const dmcr_bounds *bounds,
                        const dmcr_opt *opt, float *phi, void *ws, size_t ws_bytes, hipStream_t st, Plan &p,
                        Solver **out, std::vector<char> &mem)
{
    if (!opt_ok(opt) || !bounds || !S_target || !phi || !aligned8(phi) || !aligned8(S_target)) return DMCR_EINVAL;
    if (bounds->mode < DMCR_BOUNDS_NONE || bounds->mode > DMCR_BOUNDS_PENALTY) return DMCR_EINVAL;
    if (bounds->mode != DMCR_BOUNDS_NONE && !(bounds->lo < bounds->hi)) return DMCR_EINVAL;
    if (bounds->mode == DMCR_BOUNDS_PENALTY && !(bounds->kappa >= 0.0)) return DMCR_EINVAL;
    dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    const RLayout r = r_layout(p, *opt);
    if (ws_bytes < r.bytes) return DMCR_ENOMEM;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign)) return DMCR_EINVAL;
    mem.resize(sizeof(Solver));
    Solver *sv = new (mem.data()) Solver{p, *bounds, *opt, S_target, r, Ws{static_cast<char *>(ws)}, st, batch,
                                         opt->m, (int64_t)p.C * p.lv[0].N, dim3(), dim3(), false, false, 0.f, 0.f,
                                         0.0, *spec, Ws{static_cast<char *>(ws)}};
    sv->vg = dim3(vblocks(sv->n), batch);
    sv->sg = dim3((batch + 63) / 64);
    sv->project = bounds->mode == DMCR_BOUNDS_PROJECT;
    sv->penalty = bounds->mode == DMCR_BOUNDS_PENALTY;
    sv->lo = (float)bounds->lo;
    sv->hi = (float)bounds->hi;
    sv->invN = 1.0 / (double)p.lv[0].N;
    *out = sv;
    return DMCR_OK;
}

// Sequential coarse-to-fine schedule (the earlier multigrid practice that
// Sec. 3.3 contrasts with): reconstruct the coarsest level alone against its own
// part of the target, upsample the result (nearest neighbour) as the start of
// the next finer level, and so on down to the finest field.  Stage s uses the
// single-level spec of level s; its target is the level-s slice of the
// multigrid target (the descriptor is level-major).
struct C2FLayout {
    size_t tgt;        // [B][max K_s] double
    size_t stage_ws;   // workspace of the stage solvers
    size_t E;          // [B] double (final multigrid error)
    size_t grad;       // [B][C][N] float (final evaluation)
    size_t bytes;
};

dmcr_spec stage_spec(const dmcr_spec &s, const Plan &p, int l)
{
    dmcr_spec t = s;
    for (int a = 0; a < p.ndim; ++a) t.shape[a] = s.shape[a] >> l;
    t.n_levels = 1;
    t.max_disp[0] = s.max_disp[l];
    t.level_weight[0] = 1.0;
    return t;
}

dmcr_status c2f_layout(const dmcr_spec *spec, int B, const dmcr_opt &o, const Plan &p, C2FLayout *out)
{
    C2FLayout c{};
    size_t top = align_up_bytes(p.bytes);
    int64_t kmax = 0;
    size_t wsmax = 0;
    for (int l = 0; l < p.L; ++l) {
        kmax = std::max<int64_t>(kmax, p.lvl_off[l + 1] - p.lvl_off[l]);
        const dmcr_spec t = stage_spec(*spec, p, l);
        Plan ps;
        dmcr_status st = make_plan(&t, B, &ps);
        if (st != DMCR_OK) return st;
        wsmax = std::max(wsmax, r_layout(ps, o).bytes);
    }
    c.tgt = top;
    top = align_up_bytes(top + (size_t)B * kmax * 8);
    c.stage_ws = top;
    top = align_up_bytes(top + wsmax);
    c.E = top;
    top = align_up_bytes(top + (size_t)B * 8);
    c.grad = top;
    top = align_up_bytes(top + (size_t)B * p.C * p.lv[0].N * 4);
    c.bytes = top;
    *out = c;
    return DMCR_OK;
}

}  // namespace

extern "C" {

dmcr_status dmcr_reconstruct_c2f_workspace_size(const dmcr_spec *spec, int32_t batch, const dmcr_opt *opt,
                                                size_t *bytes)
{
    if (!bytes || !opt_ok(opt)) return DMCR_EINVAL;
    Plan p;
    dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    C2FLayout c;
    if ((s = c2f_layout(spec, batch, *opt, p, &c)) != DMCR_OK) return s;
    *bytes = c.bytes;
    return DMCR_OK;
}

dmcr_status dmcr_reconstruct_coarse_to_fine(const dmcr_spec *spec, int32_t batch, const double *S_target,
                                            const dmcr_bounds *bounds, const dmcr_opt *opt, float *phi,
                                            dmcr_result *results, void *ws, size_t ws_bytes, hipStream_t st)
{
    if (!results || batch < 1 || !S_target || !phi || !bounds || !opt_ok(opt)) return DMCR_EINVAL;
    if (!aligned8(phi) || !aligned8(S_target)) return DMCR_EINVAL;
    Plan p;
    dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    C2FLayout c;
    if ((s = c2f_layout(spec, batch, *opt, p, &c)) != DMCR_OK) return s;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign)) return DMCR_EINVAL;
    if (ws_bytes < c.bytes) return DMCR_ENOMEM;
    char *base = static_cast<char *>(ws);
    const Ws w{base};
    // the pyramid of the start field: level l's start is the l-fold mean pool
    RT(run_pyramid_levels(p, phi, w, st));
    std::vector<int> iters(batch, 0), evals(batch, 0);
    std::vector<int32_t> all(batch);
    for (int b = 0; b < batch; ++b) all[b] = b;
    for (int l = p.L - 1; l >= 0; --l) {
        float *x = (l == 0) ? phi : w.at<float>(p.lv[l].field);
        if (l + 1 < p.L) RT(launch_upsample(p, l, w.at<float>(p.lv[l + 1].field), x, st));
        const int64_t Kl = p.lvl_off[l + 1] - p.lvl_off[l];
        double *tgt = w.at<double>(c.tgt);
        RT(hipMemcpy2DAsync(tgt, Kl * 8, S_target + p.lvl_off[l], p.K * 8, Kl * 8, batch, hipMemcpyDeviceToDevice,
                            st));
        const dmcr_spec t = stage_spec(*spec, p, l);
        Plan ps;
        Solver *sv = nullptr;
        std::vector<char> mem;
        s = make_solver(&t, batch, tgt, bounds, opt, x, base + c.stage_ws, c.E - c.stage_ws, st, ps, &sv, mem);
        if (s != DMCR_OK) return s;
        std::vector<dmcr_slot> slots(batch);
        dmcr_ring ring{opt->m - 1, 0};
        s = sv->start(x, all.data(), batch, slots.data());
        if (s == DMCR_OK) s = sv->iterate(x, slots.data(), &ring, opt->max_iter);
        sv->~Solver();
        if (s != DMCR_OK) return s;
        for (int b = 0; b < batch; ++b) {
            iters[b] += slots[b].iters;
            evals[b] += slots[b].evals;
        }
    }
    // the finest field against the whole multigrid target
    double *Ed = w.at<double>(c.E);
    RS(loss_grad_internal(p, phi, S_target, Ed, w.at<float>(c.grad), w, st));
    std::vector<double> hE(batch);
    RT(hipMemcpyAsync(hE.data(), Ed, batch * sizeof(double), hipMemcpyDeviceToHost, st));
    RT(hipStreamSynchronize(st));
    bool all_ok = true;
    for (int b = 0; b < batch; ++b) {
        results[b].final_E = hE[b];
        results[b].final_derr = hE[b];
        results[b].iters = iters[b];
        results[b].evals = evals[b] + 1;
        results[b].why = !std::isfinite(hE[b]) ? DMCR_ENONFINITE : (hE[b] <= opt->tol_derr ? DMCR_OK : DMCR_NOT_CONVERGED);
        all_ok &= results[b].why == DMCR_OK;
    }
    return all_ok ? DMCR_OK : DMCR_NOT_CONVERGED;
}

dmcr_status dmcr_penalised_loss_grad(const dmcr_spec *spec, int32_t batch, const float *phi, const double *S_target,
                                     const dmcr_bounds *bounds, double *L, double *E, float *grad, void *ws,
                                     size_t ws_bytes, hipStream_t stream)
{
    if (!bounds || !L || !phi || !S_target || !E || !grad) return DMCR_EINVAL;
    if (bounds->mode < DMCR_BOUNDS_NONE || bounds->mode > DMCR_BOUNDS_PENALTY) return DMCR_EINVAL;
    if (bounds->mode == DMCR_BOUNDS_PENALTY && (!(bounds->lo < bounds->hi) || !(bounds->kappa >= 0.0)))
        return DMCR_EINVAL;
    if (!aligned8(phi) || !aligned8(grad) || !aligned8(S_target) || !aligned8(E) || !aligned8(L)) return DMCR_EINVAL;
    Plan p;
    dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    if (ws_bytes < p.bytes) return DMCR_ENOMEM;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign)) return DMCR_EINVAL;
    const Ws w{static_cast<char *>(ws)};
    RS(loss_grad_internal(p, phi, S_target, E, grad, w, stream));
    const double *Ebc = nullptr;
    if (bounds->mode == DMCR_BOUNDS_PENALTY) {
        const int64_t n = (int64_t)p.C * p.lv[0].N;
        const double invN = 1.0 / (double)p.lv[0].N;
        const float lo = (float)bounds->lo, hi = (float)bounds->hi;
        double *part = w.at<double>(p.Pen);
        double *ebc = part + (int64_t)p.B * p.pen_blocks;
        hipLaunchKernelGGL(k_pen_part, dim3(p.pen_blocks, batch), dim3(kV), 0, stream, phi, n, invN, lo, hi, part,
                           p.pen_blocks);
        hipLaunchKernelGGL(k_sum_parts, dim3(batch), dim3(kV), 0, stream, (const double *)part, p.pen_blocks, ebc,
                           batch);
        hipLaunchKernelGGL(k_pen_grad, dim3(vblocks(n), batch), dim3(kV), 0, stream, phi, grad, (const double *)E,
                           bounds->kappa, n, invN, lo, hi);
        Ebc = ebc;
    }
    hipLaunchKernelGGL(k_pen_loss, dim3((batch + 63) / 64), dim3(64), 0, stream, (const double *)E, Ebc, bounds->kappa,
                       L, batch);
    RT(hipGetLastError());
    return DMCR_OK;
}

dmcr_status dmcr_reconstruct_workspace_size(const dmcr_spec *spec, int32_t batch, const dmcr_opt *opt,
                                            size_t *bytes)
{
    if (!bytes || !opt_ok(opt)) return DMCR_EINVAL;
    Plan p;
    dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    *bytes = r_layout(p, *opt).bytes;
    return DMCR_OK;
}

dmcr_status dmcr_solver_start(const dmcr_spec *spec, int32_t batch, const int32_t *which, int32_t nwhich,
                              const double *S_target, const dmcr_bounds *bounds, const dmcr_opt *opt, float *phi,
                              dmcr_slot *slots, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!which || !slots || nwhich < 0) return DMCR_EINVAL;
    for (int i = 0; i < nwhich; ++i)
        if (which[i] < 0 || which[i] >= batch) return DMCR_EINVAL;
    Plan p;
    Solver *sv = nullptr;
    std::vector<char> mem;
    dmcr_status s = make_solver(spec, batch, S_target, bounds, opt, phi, ws, ws_bytes, stream, p, &sv, mem);
    if (s != DMCR_OK) return s;
    s = sv->start(phi, which, nwhich, slots);
    sv->~Solver();
    return s;
}

dmcr_status dmcr_solver_iterate(const dmcr_spec *spec, int32_t batch, const double *S_target,
                                const dmcr_bounds *bounds, const dmcr_opt *opt, float *phi, dmcr_slot *slots,
                                dmcr_ring *ring, int32_t iterations, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!slots || !ring || !opt || iterations < 0 || ring->count < 0 || ring->count > opt->m || ring->head < 0 ||
        ring->head >= opt->m)
        return DMCR_EINVAL;
    Plan p;
    Solver *sv = nullptr;
    std::vector<char> mem;
    dmcr_status s = make_solver(spec, batch, S_target, bounds, opt, phi, ws, ws_bytes, stream, p, &sv, mem);
    if (s != DMCR_OK) return s;
    s = sv->iterate(phi, slots, ring, iterations);
    sv->~Solver();
    return s;
}

dmcr_status dmcr_reconstruct(const dmcr_spec *spec, int32_t batch, const double *S_target, const dmcr_bounds *bounds,
                             const dmcr_opt *opt, float *phi, dmcr_result *results, void *ws, size_t ws_bytes,
                             hipStream_t st)
{
    if (!results || batch < 1) return DMCR_EINVAL;
    Plan p;
    Solver *sv = nullptr;
    std::vector<char> mem;
    dmcr_status s = make_solver(spec, batch, S_target, bounds, opt, phi, ws, ws_bytes, st, p, &sv, mem);
    if (s != DMCR_OK) return s;
    std::vector<dmcr_slot> slots(batch);
    std::vector<int32_t> all(batch);
    for (int b = 0; b < batch; ++b) all[b] = b;
    dmcr_ring ring{opt->m - 1, 0};
    s = sv->start(phi, all.data(), batch, slots.data());
    if (s == DMCR_OK) s = sv->iterate(phi, slots.data(), &ring, opt->max_iter);
    sv->~Solver();
    if (s != DMCR_OK) return s;
    bool all_ok = true;
    for (int b = 0; b < batch; ++b) {
        results[b].final_E = slots[b].E;
        results[b].final_derr = slots[b].E;
        results[b].iters = slots[b].iters;
        results[b].evals = slots[b].evals;
        results[b].why = slots[b].status == DMCR_RUNNING ? DMCR_NOT_CONVERGED : slots[b].status;
        all_ok &= results[b].why == DMCR_OK;
    }
    return all_ok ? DMCR_OK : DMCR_NOT_CONVERGED;
}

}  // extern "C"
