// C ABI of libdmcr: validation, planning (level shapes, displacement sets,
// descriptor layout, workspace carving, path choice) and the launch order of
// the forward, error and adjoint stages.  See include/dmcr.h for the contract.
#include <string.h>

#include <algorithm>
#include <cmath>

#include "dmcr_internal.h"

namespace dmcr {

bool fft_supported(const Plan &p, int l);

namespace {

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Carver {
    size_t top = 0;
    size_t take(size_t bytes)
    {
        const size_t at = top;
        top = align_up(top + bytes);
        return at;
    }
};

// Rough per-level cost model used by DMCR_PATH_AUTO (seconds per field).  It
// depends on the shape only, never on the batch size, so that a field takes the
// same kernels (and rounds the same way) alone and in any batch.
double direct_cost(const Plan &p, int l)
{
    const LevelPlan &L = p.lv[l];
    double macs = 0;
    for (int q = 0; q < p.npairs; ++q) macs += (double)L.N * (double)L.cnt[q];
    double vol = 1;
    for (int d = 0; d < p.ndim; ++d) vol *= L.box;
    macs += (double)L.N * vol * p.C * p.C;  // adjoint
    return macs / 4.0e12 + 3 * 4e-6;
}

double fft_cost(const Plan &p, int l)
{
    const LevelPlan &L = p.lv[l];
    const double bytes = (double)p.C * L.N * 60.0;
    return bytes / 4.0e12 + (p.ndim == 3 ? 12 : 8) * 4e-6;
}

}  // namespace

dmcr_status make_plan(const dmcr_spec *s, int B, Plan *pp)
{
    if (!s || !pp) return DMCR_EINVAL;
    Plan &p = *pp;
    memset(&p, 0, sizeof(Plan));
    if (s->ndim != 2 && s->ndim != 3) return DMCR_EUNSUPPORTED;
    if (B < 1) return DMCR_EINVAL;
    p.ndim = s->ndim;
    p.B = B;
    if (s->n_channels < 1 || s->n_channels > kMaxChannels) return DMCR_EINVAL;
    p.C = s->n_channels;
    if (s->n_levels < 0 || s->n_levels > kMaxLevels) return DMCR_EINVAL;
    int minax0 = 1 << 30;
    for (int a = 0; a < p.ndim; ++a) {
        if (!is_pow2(s->shape[a]) || s->shape[a] < 2) return DMCR_EUNSUPPORTED;
        minax0 = std::min(minax0, s->shape[a]);
    }
    // n_levels = 0: the level rule of Appendix B (P = 31 gives 1, 2, 3 levels at 64,
    // 128, 256), i.e. levels down to a coarsest side of about 2 (P + 1), P = max_disp[0]
    const bool rule = s->n_levels == 0;
    if (rule) {
        if (s->max_disp[0] < 0) return DMCR_EINVAL;
        const double lv = std::log2((double)minax0 / (2.0 * (s->max_disp[0] + 1.0)));
        p.L = std::max(1, std::min(kMaxLevels, 1 + (int)std::lround(lv)));
        while (p.L > 1 && (minax0 >> (p.L - 1)) < 2) --p.L;
    } else {
        p.L = s->n_levels;
    }
    for (int a = 0; a < p.ndim; ++a) {
        if ((s->shape[a] >> (p.L - 1)) < 2) return DMCR_EINVAL;
        p.shape[a] = s->shape[a];
    }
    if (p.ndim == 2) p.shape[2] = 1;
    if (s->flags & ~(DMCR_FLAG_RECOMPUTE | DMCR_FLAG_FUSED_PLANES)) return DMCR_EINVAL;
    p.flags = s->flags;
    if (s->path < DMCR_PATH_AUTO || s->path > DMCR_PATH_DIRECT) return DMCR_EINVAL;
    // descriptor kind and soft-threshold constants (Sec. 3.2.4): the inflection
    // condition f''(0.75) = 0 gives c2 = -0.75, then f(0) = 0 and f(1) = 1 fix c1, c3
    if (s->descriptor < DMCR_DESC_S2 || s->descriptor > DMCR_DESC_STILDE || s->s3_max_disp < 0) return DMCR_EINVAL;
    p.desc = s->descriptor;
    p.s3 = s->s3_max_disp > 0;
    if (p.desc != DMCR_DESC_S2) {
        p.alpha = (s->alpha == 0.0) ? 10.0 : s->alpha;
        if (!(p.alpha > 0.0) || !std::isfinite(p.alpha)) return DMCR_EINVAL;
        if (s->path == DMCR_PATH_FFT) return DMCR_EUNSUPPORTED;
        auto sig = [](double z) { return 1.0 / (1.0 + std::exp(-z)); };
        p.c2 = -0.75;
        const double lo = sig(p.alpha * p.c2), hi = sig(p.alpha * (1.0 + p.c2));
        p.c1 = 1.0 / (hi - lo);
        p.c3 = -p.c1 * lo;
        const double fh = p.c1 * sig(p.alpha * (0.5 + p.c2)) + p.c3;
        p.fh = fh;
        p.F = fh * fh;
    }
    // pairs
    if (s->n_pairs <= 0) {
        for (int i = 0; i < p.C; ++i)
            for (int j = i; j < p.C; ++j) {
                p.pi[p.npairs] = i;
                p.pj[p.npairs] = j;
                ++p.npairs;
            }
    } else {
        if (s->n_pairs > kMaxPairs) return DMCR_EINVAL;
        p.npairs = s->n_pairs;
        for (int q = 0; q < p.npairs; ++q) {
            const int i = s->pairs[2 * q], j = s->pairs[2 * q + 1];
            if (i < 0 || j < i || j >= p.C) return DMCR_EINVAL;
            for (int r = 0; r < q; ++r)
                if (p.pi[r] == i && p.pj[r] == j) return DMCR_EINVAL;
            p.pi[q] = i;
            p.pj[q] = j;
        }
    }
    if (p.desc == DMCR_DESC_STILDE) {
        // the map of pair (i, j) reads the r = 0 entries of the auto pairs (i, i) and
        // (j, j); the three-point map reads the auto pair of every channel
        auto has_auto = [&](int c) {
            for (int r = 0; r < p.npairs; ++r)
                if (p.pi[r] == c && p.pj[r] == c) return true;
            return false;
        };
        for (int q = 0; q < p.npairs; ++q)
            if (!has_auto(p.pi[q]) || !has_auto(p.pj[q])) return DMCR_EINVAL;
        if (p.s3)
            for (int c = 0; c < p.C; ++c)
                if (!has_auto(c)) return DMCR_EINVAL;
    }
    // levels
    int64_t off = 0;
    p.Z = 0;
    for (int l = 0; l < p.L; ++l) {
        LevelPlan &L = p.lv[l];
        int minax = 1 << 30;
        L.N = 1;
        for (int a = 0; a < 3; ++a) {
            L.n[a] = (a < p.ndim) ? (p.shape[a] >> l) : 1;
            L.N *= L.n[a];
            if (a < p.ndim) minax = std::min(minax, L.n[a]);
        }
        // P_l = min(P, n_l / 2 - 1): larger displacements would alias on the level
        const int Pl = s->max_disp[rule ? 0 : l];
        if (Pl < 0) return DMCR_EINVAL;
        L.P = std::min(Pl, minax / 2 - 1);
        L.box = 2 * L.P + 1;
        L.h = L.n[p.ndim - 1] / 2 + 1;
        L.hp = (L.n[p.ndim - 1] >= 32) ? (L.h + 15) / 16 * 16 : L.h;
        // w_l (eq. mg): 0 selects 2^{d l / 2} (level 0 finest), the square root of
        // the fine voxels one coarse voxel summarises (the footnote's 2^{l-1} in 2-D)
        const double wl = rule ? 0.0 : s->level_weight[l];
        if (wl == 0.0)
            p.w[l] = std::pow(2.0, 0.5 * p.ndim * l);
        else if (wl > 0.0 && std::isfinite(wl))
            p.w[l] = wl;
        else
            return DMCR_EINVAL;
        int64_t vol = 1;
        for (int a = 0; a < p.ndim; ++a) vol *= L.box;
        p.lvl_off[l] = off;
        int64_t lvlK = 0;
        for (int q = 0; q < p.npairs; ++q) {
            L.off[q] = off;
            L.cnt[q] = (p.pi[q] == p.pj[q]) ? (vol + 1) / 2 : vol;
            off += L.cnt[q];
            lvlK += L.cnt[q];
        }
        if (p.s3) {
            L.s3P = std::min(s->s3_max_disp, L.P);
            if (p.desc == DMCR_DESC_STILDE && 2 * L.s3P > L.P) return DMCR_EINVAL;  // map reads S2(r_a - r_b)
            L.s3M = 1;
            for (int a = 0; a < p.ndim; ++a) L.s3M *= 2 * L.s3P + 1;
            L.s3K = (int64_t)L.s3M * (L.s3M + 1) / 2;
            L.s3off = off;
            off += p.C * L.s3K;
            lvlK += p.C * L.s3K;
        }
        p.Z += p.w[l] * p.w[l] * (double)lvlK;
    }
    p.lvl_off[p.L] = off;
    p.K = off;
    // path per level
    for (int l = 0; l < p.L; ++l) {
        LevelPlan &L = p.lv[l];
        int tile[3];
        const bool dok = direct_supported(p, l, tile);
        const bool fok = fft_supported(p, l);
        if (s->path == DMCR_PATH_DIRECT || p.desc != DMCR_DESC_S2) {
            if (!dok) return DMCR_EUNSUPPORTED;
            L.path = DMCR_PATH_DIRECT;
        } else if (s->path == DMCR_PATH_FFT) {
            if (!fok) return DMCR_EUNSUPPORTED;
            L.path = DMCR_PATH_FFT;
        } else {
            if (!dok && !fok) return DMCR_EUNSUPPORTED;
            L.path = (dok && (!fok || direct_cost(p, l) < fft_cost(p, l))) ? DMCR_PATH_DIRECT : DMCR_PATH_FFT;
        }
        if (dok) {
            L.tile[0] = tile[0];
            L.tile[1] = tile[1];
            L.tile[2] = tile[2];
            L.n_tiles = (L.N / ((int64_t)tile[0] * tile[1] * tile[2]));
        }
    }
    if (p.s3)
        for (int l = 0; l < p.L; ++l) {
            LevelPlan &L = p.lv[l];
            if (!s3_configure(p, l)) return DMCR_EUNSUPPORTED;
        }
    // workspace
    Carver cv;
    const int C = p.C;
    for (int l = 0; l < p.L; ++l) {
        LevelPlan &L = p.lv[l];
        const int64_t field = (int64_t)B * C * L.N;
        if (l > 0) {
            L.field = cv.take(field * sizeof(float));
            L.grad = cv.take(field * sizeof(float));
        }
        int64_t vol = 1;
        for (int a = 0; a < p.ndim; ++a) vol *= L.box;
        if (L.path == DMCR_PATH_DIRECT) L.KB0 = cv.take((size_t)B * C * C * vol * sizeof(float));
        if (L.path == DMCR_PATH_FFT) {
            const int64_t nl = L.n[p.ndim - 1];
            const int64_t half = L.N / nl * L.hp;  // complex entries of one (padded) half spectrum
            L.X = cv.take((size_t)B * C * half * sizeof(float2));
            L.mparts = fft_mean_parts(p, l);
            L.msum = cv.take((size_t)B * C * L.mparts * sizeof(double));
            L.mu = cv.take((size_t)B * C * sizeof(double));
            const int64_t inner = half / L.n[0];
            L.Y = cv.take((size_t)B * p.npairs * L.box * inner * sizeof(float2));
            if (p.ndim == 3) {
                L.Y2 = cv.take((size_t)B * p.npairs * L.box * L.box * L.hp * sizeof(float2));
                L.KB1 = cv.take((size_t)B * C * C * L.box * L.box * L.hp * sizeof(float2));
                L.KB2 = cv.take((size_t)B * C * C * L.box * L.n[1] * L.hp * sizeof(float2));
            } else {
                L.KB1 = cv.take((size_t)B * C * C * L.box * L.hp * sizeof(float2));
            }
        } else {
            int64_t kmax = 0;
            for (int q = 0; q < p.npairs; ++q) kmax = std::max(kmax, L.cnt[q]);
            L.part = cv.take((size_t)B * p.npairs * L.n_tiles * kmax * sizeof(double));
        }
    }
    if (p.s3)
        for (int l = 0; l < p.L; ++l) {
            LevelPlan &L = p.lv[l];
            L.s3part = cv.take((size_t)B * C * L.s3chunks * L.s3K * sizeof(float));
            L.s3Q = cv.take((size_t)B * C * L.s3M * L.N * sizeof(float));
            L.s3G = cv.take((size_t)B * C * L.s3Kp * L.s3Mp * sizeof(float));
            if (p.desc == DMCR_DESC_S2 && !L.s3mf) L.s3R = cv.take((size_t)B * C * L.s3M * L.N * sizeof(float));
        }
    p.S = cv.take((size_t)B * p.K * sizeof(float));
    p.G = cv.take((size_t)B * p.K * sizeof(float));
    p.err_chunks = std::max<int64_t>(1, std::min<int64_t>(8192, (p.K + 511) / 512));
    p.Epart = cv.take((size_t)B * p.err_chunks * sizeof(double));
    p.pen_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(2048, ((int64_t)C * p.lv[0].N + 1023) / 1024));
    p.Pen = cv.take((size_t)B * (p.pen_blocks + 1) * sizeof(double));
    p.bytes = cv.top;
    return DMCR_OK;
}

namespace {

dmcr_status dev(hipError_t e) { return e == hipSuccess ? DMCR_OK : DMCR_EDEVICE; }

#define DMCR_TRY(expr)                                  \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return DMCR_EDEVICE;      \
    } while (0)

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

dmcr_status check_ws(const Plan &p, void *ws, size_t ws_bytes)
{
    if (ws_bytes < p.bytes) return DMCR_ENOMEM;
    if (p.bytes > 0 && (!ws || !aligned(ws))) return DMCR_EINVAL;
    return DMCR_OK;
}

const float *level_field(const Plan &p, int l, const float *phi, const Ws &ws)
{
    return l == 0 ? phi : ws.at<const float>(p.lv[l].field);
}

// levels 1..L-1 of the pyramid of phi into out[1..L-1]
hipError_t pyramid_into(const Plan &p, const float *phi, float *const *out, hipStream_t st)
{
    for (int l = 0; l + 1 < p.L;) {
        const float *f = (l == 0) ? phi : out[l];
        hipError_t e;
        // two levels per pass (its float4 loads need a 16-byte aligned field; the
        // caller's field may be a view that is only 8-byte aligned)
        if (l + 2 < p.L && reinterpret_cast<uintptr_t>(f) % 16 == 0) {
            e = launch_restrict2(p, l, f, out[l + 1], out[l + 2], st);
            l += 2;
        } else {
            e = launch_restrict(p, l, f, out[l + 1], st);
            l += 1;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t run_pyramid(const Plan &p, const float *phi, const Ws &ws, hipStream_t st)
{
    float *out[kMaxLevels] = {};
    for (int l = 1; l < p.L; ++l) out[l] = ws.at<float>(p.lv[l].field);
    return pyramid_into(p, phi, out, st);
}

// Internal streams that let independent work of one call overlap: the levels
// of the pyramid run on their own lanes, and a recomputed spectrum is built on
// a side lane while the caller's stream finishes the forward and builds the
// cotangent transforms.  Every lane joins the caller's stream before the call
// returns, so the caller sees ordinary stream semantics.  Pools are per host
// thread and per device, so concurrent callers never share an event; each is
// created on its first use and kept until the process ends.
struct Lanes {
    static constexpr int kSide = 3;
    static constexpr int kEvents = 96;
    bool ready = false;
    hipStream_t side[kSide] = {};
    hipEvent_t ev[kEvents] = {};
    int next = 0;

    // on the current device; a failure destroys what it created, so a later call
    // starts again from nothing
    hipError_t init()
    {
        if (ready) return hipSuccess;
        hipError_t e = hipSuccess;
        int ns = 0, ne = 0;
        for (; ns < kSide && e == hipSuccess; ++ns)
            if ((e = hipStreamCreateWithFlags(&side[ns], hipStreamNonBlocking)) != hipSuccess) break;
        for (; e == hipSuccess && ne < kEvents; ++ne)
            if ((e = hipEventCreateWithFlags(&ev[ne], hipEventDisableTiming)) != hipSuccess) break;
        if (e != hipSuccess) {
            for (int i = 0; i < ne; ++i) (void)hipEventDestroy(ev[i]);
            for (int i = 0; i < ns; ++i) (void)hipStreamDestroy(side[i]);
            return e;
        }
        ready = true;
        return hipSuccess;
    }
    hipEvent_t event() { return ev[next++ % kEvents]; }
};

constexpr int kMaxDevices = 16;
thread_local Lanes tl_lanes[kMaxDevices];

// this thread's lanes on the current device
hipError_t lanes_here(Lanes **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if ((e = tl_lanes[dev].init()) != hipSuccess) return e;
    *out = &tl_lanes[dev];
    return hipSuccess;
}

struct Sched {
    Lanes *ln;
    hipStream_t main;
    bool multi;  // false: everything on the caller's stream
    bool side_recompute;  // a recomputed spectrum is built on a spare lane
    hipStream_t lane(int l) const { return (l == 0 || !multi) ? main : ln->side[(l - 1) % Lanes::kSide]; }
    // a stream that is not lane(l) of a level in use, for level l's recompute
    hipStream_t spare(int l, int L) const
    {
        if (!multi) return main;
        if (L == 1) return ln->side[0];
        return (l == 0) ? ln->side[(L - 1) % Lanes::kSide] : main;
    }
    hipError_t join(hipStream_t to, hipStream_t from)
    {
        if (to == from || !multi) return hipSuccess;
        hipEvent_t e = ln->event();
        hipError_t r = hipEventRecord(e, from);
        if (r != hipSuccess) return r;
        return hipStreamWaitEvent(to, e, 0);
    }
};

// Side lanes pay off only when the passes are long enough to hide the extra
// event waits; smaller batches stay on the caller's stream (measured: 2-D 512^2
// three-level evaluations of 1, 4 and 16 fields are faster on one stream,
// 256^3 and 64 x 512^2 (16.8M voxels) with lanes; the two-channel 128^3
// three-level evaluation took 0.167-0.215 ms with lanes, varying between
// processes, against a steady 0.199 ms on one stream).  The
// soft-threshold and three-point levels are long ALU- or matrix-bound kernels
// whose coarse levels fill only part of the chip, so their levels always run side
// by side.  Under stream
// capture the event waits become graph edges that cost no host time, so a
// captured call also runs its levels side by side (measured: the two-channel
// 128^3 three-level evaluation replays in 0.139 ms with lanes and takes
// 0.193 ms eager on one stream).  A recompute moves to a spare lane only by the
// size rule and only for one level: there it takes the two-pass spectrum, and
// results must not depend on capture.  With several levels each level recomputes
// its spectrum on its own lane (an eager batch of two 128^3 three-level fields on
// lanes with the recomputes on spare lanes gave a gradient that differed between
// two calls, cause not found; that schedule is not used).
constexpr int64_t kLaneMinVoxels = int64_t(1) << 24;

hipError_t make_sched(const Plan &p, hipStream_t st, Sched *s)
{
    // the null stream cannot be captured
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (st != nullptr) {
        hipError_t e = hipStreamIsCapturing(st, &cs);
        if (e != hipSuccess) return e;
    }
    const bool eager_multi = (int64_t)p.B * p.C * p.lv[0].N >= kLaneMinVoxels ||
                             ((p.desc != DMCR_DESC_S2 || p.s3) && p.L > 1);
    const bool multi = eager_multi || (cs == hipStreamCaptureStatusActive && p.L > 1);
    Lanes *ln = nullptr;   // dereferenced only when multi
    if (multi) {
        hipError_t e = lanes_here(&ln);
        if (e != hipSuccess) return e;
        ln->next = 0;
    }
    *s = Sched{ln, st, multi, eager_multi && p.L == 1};
    return hipSuccess;
}

// Forward of every level on its lane.  x_free[l] (recompute only) marks the
// point after which level l's partial spectrum may be overwritten.
hipError_t run_forward(const Plan &p, const float *phi, float *S, const Ws &ws, Sched &sc,
                       hipEvent_t *x_free = nullptr)
{
    hipError_t e = run_pyramid(p, phi, ws, sc.main);
    if (e != hipSuccess) return e;
    for (int l = 1; l < p.L; ++l)
        if ((e = sc.join(sc.lane(l), sc.main)) != hipSuccess) return e;
    for (int l = 0; l < p.L; ++l) {
        const float *f = level_field(p, l, phi, ws);
        e = (p.lv[l].path == DMCR_PATH_FFT)
                ? fft_forward_level(p, l, f, S, ws, sc.lane(l), x_free ? x_free[l] : nullptr)
                : direct_forward_level(p, l, f, S, ws, sc.lane(l));
        if (e != hipSuccess) return e;
        if (p.s3 && (e = s3_forward_level(p, l, f, S, ws, sc.lane(l))) != hipSuccess) return e;
    }
    for (int l = 1; l < p.L; ++l)
        if ((e = sc.join(sc.main, sc.lane(l))) != hipSuccess) return e;
    if (p.desc == DMCR_DESC_STILDE) {
        if ((e = launch_stilde(p, S, sc.main)) != hipSuccess) return e;
        if (p.s3) return launch_s3_map(p, S, sc.main);
    }
    return hipSuccess;
}

// Adjoint of every level on its lane, coarsest first: each level's total
// gradient is its own term plus the prolongation of the next coarser total
// (Sec. 3.3: back-propagation through all levels at once), added on the level's
// lane once the coarser total is complete; where the level ends in the
// contiguous-axis inverse, that pass adds it while writing.
hipError_t run_adjoint(const Plan &p, const float *phi, const float *G, float *grad, bool have_spectrum,
                       const Ws &ws, Sched &sc, hipEvent_t *x_free = nullptr, const double *St = nullptr)
{
    hipError_t e;
    // with St each level forms its cotangent from its own S on its own lane, so
    // the lanes need not wait for the error on the caller's stream
    if (!St)
        for (int l = 1; l < p.L; ++l)
            if ((e = sc.join(sc.lane(l), sc.main)) != hipSuccess) return e;
    // ready[l]: level l's total gradient is complete on lane(l)
    hipEvent_t ready[kMaxLevels] = {};
    for (int l = p.L - 1; l >= 0; --l) {
        const float *f = level_field(p, l, phi, ws);
        float *g = (l == 0) ? grad : ws.at<float>(p.lv[l].grad);
        const float *cg = (l + 1 < p.L) ? ws.at<float>(p.lv[l + 1].grad) : nullptr;
        hipEvent_t cready = (cg && sc.lane(l) != sc.lane(l + 1)) ? ready[l + 1] : nullptr;
        // the prolongation of the coarser total rides on the level's last inverse pass
        const bool fuse = cg && fft_fused_prolong(p, l);
        if (p.lv[l].path == DMCR_PATH_FFT) {
            const float *fc = fuse ? cg : nullptr;
            hipEvent_t fr = fuse ? cready : nullptr;
            if (!have_spectrum && x_free)
                e = fft_adjoint_level(p, l, f, G, g, false, ws, sc.lane(l), sc.spare(l, p.L), x_free[l],
                                      sc.ln->event(), St, fc, fr);
            else
                e = fft_adjoint_level(p, l, f, G, g, have_spectrum, ws, sc.lane(l), nullptr, nullptr, nullptr, St,
                                      fc, fr);
        } else {
            e = direct_adjoint_level(p, l, f, G, g, ws, sc.lane(l), St);
        }
        if (e != hipSuccess) return e;
        if (p.s3 && (e = s3_adjoint_level(p, l, f, G, g, ws, sc.lane(l), St)) != hipSuccess) return e;
        if (cg && !fuse) {
            if (cready && (e = hipStreamWaitEvent(sc.lane(l), cready, 0)) != hipSuccess) return e;
            if ((e = launch_prolong_add(p, l, cg, g, sc.lane(l))) != hipSuccess) return e;
        }
        if (l > 0 && sc.multi) {
            ready[l] = sc.ln->event();
            if ((e = hipEventRecord(ready[l], sc.lane(l))) != hipSuccess) return e;
        }
    }
    // lane(0) is the caller's stream; it waited for level 1's total, which waited
    // for level 2's, and so on, so every lane has joined it
    return hipSuccess;
}

}  // namespace

hipError_t run_pyramid_levels(const Plan &p, const float *phi, const Ws &ws, hipStream_t st)
{
    return run_pyramid(p, phi, ws, st);
}

// forward, error, adjoint with one plan (shared by dmcr_loss_grad and the
// reconstruction loop)
dmcr_status loss_grad_internal(const Plan &p, const float *phi, const double *St, double *E, float *grad,
                               const Ws &w, hipStream_t st, bool lanes)
{
    float *S = w.at<float>(p.S);
    float *G = w.at<float>(p.G);
    Sched sc;
    if (lanes)
        DMCR_TRY(make_sched(p, st, &sc));
    else
        sc = Sched{nullptr, st, false, false};
    const bool keep = (p.flags & DMCR_FLAG_RECOMPUTE) == 0;
    hipEvent_t x_free[kMaxLevels] = {};
    if (!keep && sc.side_recompute)
        for (int l = 0; l < p.L; ++l) x_free[l] = sc.ln->event();
    hipEvent_t *xf = (!keep && sc.side_recompute) ? x_free : nullptr;
    DMCR_TRY(run_forward(p, phi, S, w, sc, xf));
    // The final error sum runs on a side lane that the levels leave free: with one
    // level side lane 1 (lane 0 is the caller's stream, the recompute uses side
    // lane 0), with two or three levels side lane 2 (levels 1 and 2 take side
    // lanes 0 and 1; a three-level recompute queues behind it there).
    hipStream_t fin = st;
    if (sc.multi && p.L == 1)
        fin = sc.ln->side[1];
    else if (sc.multi && p.L <= 3)
        fin = sc.ln->side[2];
    // Product or soft descriptor (not the Appendix A map, which mixes the blocks):
    // every level's cotangent-kernel passes, two- and three-point, form its G
    // from its own S and St, so the whole error reduction moves to that side lane
    // and each level's adjoint starts right after its own forward, on its own lane.
    const bool g_inline = fin != st && (p.desc == DMCR_DESC_S2 || p.desc == DMCR_DESC_SBAR);
    if (g_inline) {
        DMCR_TRY(sc.join(fin, st));
        DMCR_TRY(launch_error(p, S, St, E, G, w, fin, fin, nullptr));
        DMCR_TRY(run_adjoint(p, phi, S, grad, keep, w, sc, xf, St));
        return dev(sc.join(st, fin));
    }
    DMCR_TRY(launch_error(p, S, St, E, G, w, st, fin, fin != st ? sc.ln->event() : nullptr));
    if (p.desc == DMCR_DESC_STILDE) {
        if (p.s3) DMCR_TRY(launch_s3_map_adjoint(p, G, st));
        DMCR_TRY(launch_stilde_adjoint(p, G, G, st));
    }
    DMCR_TRY(run_adjoint(p, phi, G, grad, keep, w, sc, xf));
    return dev(sc.join(st, fin));
}

}  // namespace dmcr

using namespace dmcr;

extern "C" {

int32_t dmcr_level_count(const dmcr_spec *spec)
{
    Plan p;
    const dmcr_status s = make_plan(spec, 1, &p);
    return s == DMCR_OK ? p.L : (int32_t)s;
}

int64_t dmcr_descriptor_size(const dmcr_spec *spec)
{
    Plan p;
    const dmcr_status s = make_plan(spec, 1, &p);
    return s == DMCR_OK ? p.K : (int64_t)s;
}

dmcr_status dmcr_descriptor_offsets(const dmcr_spec *spec, int64_t *offsets)
{
    if (!offsets) return DMCR_EINVAL;
    Plan p;
    const dmcr_status s = make_plan(spec, 1, &p);
    if (s != DMCR_OK) return s;
    int i = 0;
    for (int l = 0; l < p.L; ++l) {
        for (int q = 0; q < p.npairs; ++q) offsets[i++] = p.lv[l].off[q];
        if (p.s3)
            for (int c = 0; c < p.C; ++c) offsets[i++] = p.lv[l].s3off + c * p.lv[l].s3K;
    }
    offsets[i] = p.K;
    return DMCR_OK;
}

dmcr_status dmcr_workspace_size(const dmcr_spec *spec, int32_t batch, size_t *bytes)
{
    if (!bytes) return DMCR_EINVAL;
    Plan p;
    const dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    *bytes = p.bytes;
    return DMCR_OK;
}

dmcr_status dmcr_pyramid(const dmcr_spec *spec, int32_t batch, const float *phi, float *levels,
                         hipStream_t stream)
{
    Plan p;
    dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    if (!phi || (p.L > 1 && !levels)) return DMCR_EINVAL;
    if (!aligned8(phi) || !aligned8(levels)) return DMCR_EINVAL;
    float *out[kMaxLevels] = {};
    float *next = levels;
    for (int l = 1; l < p.L; ++l) {
        out[l] = next;
        next += (int64_t)p.B * p.C * p.lv[l].N;
    }
    return dev(pyramid_into(p, phi, out, stream));
}

dmcr_status dmcr_descriptor_forward(const dmcr_spec *spec, int32_t batch, const float *phi, float *S,
                                    void *ws, size_t ws_bytes, hipStream_t stream)
{
    Plan p;
    dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    if (!phi || !S || !aligned8(phi)) return DMCR_EINVAL;
    if ((s = check_ws(p, ws, ws_bytes)) != DMCR_OK) return s;
    Ws w{static_cast<char *>(ws)};
    Sched sc;
    DMCR_TRY(make_sched(p, stream, &sc));
    return dev(run_forward(p, phi, S, w, sc));
}

dmcr_status dmcr_descriptor_adjoint(const dmcr_spec *spec, int32_t batch, const float *phi, const float *dS,
                                    float *grad, void *ws, size_t ws_bytes, hipStream_t stream)
{
    Plan p;
    dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    if (!phi || !dS || !grad || !aligned8(phi) || !aligned8(grad)) return DMCR_EINVAL;
    if ((s = check_ws(p, ws, ws_bytes)) != DMCR_OK) return s;
    Ws w{static_cast<char *>(ws)};
    Sched sc;
    DMCR_TRY(make_sched(p, stream, &sc));
    DMCR_TRY(run_pyramid(p, phi, w, stream));
    if (p.desc == DMCR_DESC_STILDE) {
        float *G = w.at<float>(p.G);
        if (p.s3) {
            DMCR_TRY(hipMemcpyAsync(G, dS, (size_t)p.B * p.K * sizeof(float), hipMemcpyDeviceToDevice, stream));
            DMCR_TRY(launch_s3_map_adjoint(p, G, stream));
            DMCR_TRY(launch_stilde_adjoint(p, G, G, stream));
        } else {
            DMCR_TRY(launch_stilde_adjoint(p, dS, G, stream));
        }
        dS = G;
    }
    return dev(run_adjoint(p, phi, dS, grad, false, w, sc));
}

dmcr_status dmcr_error_cotangent(const dmcr_spec *spec, int32_t batch, const float *S, const double *S_target,
                                 double *E, float *G, void *ws, size_t ws_bytes, hipStream_t stream)
{
    Plan p;
    dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    if (!S || !S_target || !E || !G || !aligned8(S_target) || !aligned8(E)) return DMCR_EINVAL;
    if ((s = check_ws(p, ws, ws_bytes)) != DMCR_OK) return s;
    Ws w{static_cast<char *>(ws)};
    return dev(launch_error(p, S, S_target, E, G, w, stream));
}

dmcr_status dmcr_loss_grad(const dmcr_spec *spec, int32_t batch, const float *phi, const double *S_target,
                           double *E, float *grad, void *ws, size_t ws_bytes, hipStream_t stream)
{
    Plan p;
    dmcr_status s = make_plan(spec, batch, &p);
    if (s != DMCR_OK) return s;
    if (!phi || !S_target || !E || !grad) return DMCR_EINVAL;
    if (!aligned8(phi) || !aligned8(grad) || !aligned8(S_target) || !aligned8(E)) return DMCR_EINVAL;
    if ((s = check_ws(p, ws, ws_bytes)) != DMCR_OK) return s;
    Ws w{static_cast<char *>(ws)};
    return loss_grad_internal(p, phi, S_target, E, grad, w, stream);
}

const char *dmcr_status_string(dmcr_status status)
{
    switch (status) {
    case DMCR_OK: return "ok";
    case DMCR_EINVAL: return "invalid argument";
    case DMCR_ENOMEM: return "workspace too small";
    case DMCR_EUNSUPPORTED: return "problem not supported by this library";
    case DMCR_EDEVICE: return "HIP device or launch error";
    case DMCR_ENONFINITE: return "non-finite loss or gradient";
    case DMCR_NOT_CONVERGED: return "iteration budget spent before the tolerance";
    }
    return "unknown status";
}

}  // extern "C"
