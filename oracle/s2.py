"""Oracle for the differentiable multigrid two-point-correlation descriptor.

TEST INFRASTRUCTURE ONLY.  Plain, slow, FP64 CPU code that states what the
GPU path must compute; it shares no code, header, table or helper with the
product library and imports nothing from it.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may use it.

Sources in the paper (Seibert, Ambati, Rassloff, Kaestner, arXiv 2103.09686):
  * Sec. 3.1, eqs. (dMCR-Min_Prob), (L_func_dMCR): relaxed problem over real
    fields, loss = descriptor error + lambda * box penalty E^bc.
  * Sec. 3.2.1: S2^{a->b}(r), probability that r starts in a and ends in b.
  * Sec. 3.2.2: every pixel is a start point (n_r = I*J), ensemble average.
  * Sec. 3.2.3, eq. (convdef): periodic (mod) shifts; written 0-based here.
  * Sec. 3.3, eq. (mg) and its footnote: the same field at several
    resolutions, level l summarising 2^{d(l-1)} pixels, descriptors weighted
    by w_l and concatenated, all levels optimised together.
  * Appendix A, eq. (s2rfroms2rbar): with the identity threshold the
    corrected descriptor equals the product-form S2 used here.
  * Appendix B: point symmetry of the auto-correlation halves the set of
    displacement vectors; P = Q = 31 gives 1/2/3 levels at 64/128/256.
  * Sec. 3.2.4, eq. (softthreshold): the logistic soft threshold with slope
    alpha (10 in the paper) and constants fixed by f(0) = 0, f(1) = 1,
    f''(0.75) = 0; the quadratic reduction of its realisations is Sbar.
  * Appendix A, eq. (s2rfroms2rbar): the affine map from Sbar back to S2.

Readings where the paper is silent (each one is listed in the design notes):
  * level 1 is the finest; level l+1 is the 2^d mean pool of level l;
  * auto-correlations use the half box H_P (r = 0 or first non-zero
    component > 0), cross-correlations the full box B_P = [-P, P]^d;
  * descriptor order: level-major, then pair (i <= j, lexicographic), then r
    lexicographic with axis 0 slowest;
  * E is the squared weighted error divided by Z = sum_l w_l^2 K_l, so that a
    stopping threshold does not depend on the grid size;
  * the default weight generalises w_l = 2^{l-1} (2-D) to 2^{d(l-1)/2};
  * soft threshold on a cross pair (i, j): u = (phi_i(x) + phi_j(x + r)) / 2 at
    every r, r = 0 included; the Appendix A map generalises to
    S_ij(r) = (Sbar_ij(r) - f(1/2)^2 (Sbar_ii(0) + Sbar_jj(0))) / (1 - 2 f(1/2)^2),
    which is the paper's map for i = j, r != 0, and the identity for i = j, r = 0.
"""
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

from . import _native


# ----------------------------------------------------------------------------
# displacement sets and layout
# ----------------------------------------------------------------------------
def box(ndim: int, P: int) -> np.ndarray:
    """All r in [-P, P]^ndim, lexicographic with axis 0 slowest (K x ndim)."""
    axes = [np.arange(-P, P + 1)] * ndim
    grid = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.reshape(-1) for g in grid], axis=1).astype(np.int64)


def in_half(r) -> bool:
    """r = 0 or its first non-zero component is positive (point-symmetry half)."""
    for c in r:
        if c != 0:
            return c > 0
    return True


def half_box(ndim: int, P: int) -> np.ndarray:
    """The half box H_P in lexicographic order: ((2P+1)^d + 1) / 2 vectors."""
    b = box(ndim, P)
    keep = np.array([in_half(r) for r in b], dtype=bool)
    return b[keep]


def level_disp(shape, n_levels: int, P: int) -> Tuple[int, ...]:
    """P_l = min(P, min_axis(n_l) / 2 - 1) for every level (Sec. 3.3 keeps one P per
    level; a displacement longer than half the coarse grid would alias)."""
    return tuple(min(int(P), min(int(n) >> l for n in shape) // 2 - 1) for l in range(n_levels))


def all_pairs(C: int) -> List[Tuple[int, int]]:
    return [(i, j) for i in range(C) for j in range(i, C)]


# descriptor kinds: the product form S2 (the corrected descriptor of the
# identity threshold), the paper's soft-threshold Sbar, and Sbar mapped back
# by Appendix A (S~, equal to S2 on binary fields)
DESCRIPTORS = ("s2", "sbar", "stilde")


def soft_threshold_constants(alpha: float):
    """(c1, c2, c3) of f(u) = c1 / (1 + exp(-alpha (u + c2))) + c3 from the three
    conditions of Sec. 3.2.4: f''(0.75) = 0 puts the logistic's inflection at
    u = 0.75, so c2 = -0.75; f(0) = 0 and f(1) = 1 are then two linear
    equations in c1 and c3."""
    sig = lambda z: 1.0 / (1.0 + np.exp(-z))
    c2 = -0.75
    lo, hi = sig(alpha * (0.0 + c2)), sig(alpha * (1.0 + c2))
    c1 = 1.0 / (hi - lo)
    c3 = -c1 * lo
    return float(c1), float(c2), float(c3)


def soft_threshold(u, alpha: float):
    """The logistic soft threshold f(u) of eq. (softthreshold)."""
    c1, c2, c3 = soft_threshold_constants(alpha)
    return c1 / (1.0 + np.exp(-alpha * (np.asarray(u, np.float64) + c2))) + c3


@dataclass
class Spec:
    """Oracle-side statement of one multigrid descriptor."""
    shape: Tuple[int, ...]            # finest-level grid, 2 or 3 axes
    n_channels: int = 1               # explicit soft phase indicators
    n_levels: int = 1
    max_disp: Tuple[int, ...] = (16,)  # P per level (already valid for the level)
    level_weight: Tuple[float, ...] = ()
    pairs: Tuple[Tuple[int, int], ...] = ()
    descriptor: str = "s2"            # one of DESCRIPTORS
    alpha: float = 10.0               # soft-threshold slope (sbar, stilde)
    s3_max_disp: int = 0              # > 0: three-point block of every channel, vectors in [-P3, P3]^d

    def __post_init__(self):
        self.shape = tuple(int(s) for s in self.shape)
        d = len(self.shape)
        if len(self.max_disp) == 1 and self.n_levels > 1:
            self.max_disp = tuple(self.max_disp) * self.n_levels
        self.max_disp = tuple(int(p) for p in self.max_disp)
        if not self.level_weight:
            self.level_weight = tuple(2.0 ** (d * l / 2.0) for l in range(self.n_levels))
        if not self.pairs:
            self.pairs = tuple(all_pairs(self.n_channels))
        if self.descriptor not in DESCRIPTORS:
            raise ValueError("descriptor must be one of %s" % (DESCRIPTORS,))
        if self.descriptor == "stilde":
            autos = {i for (i, j) in self.pairs if i == j}
            for (i, j) in self.pairs:
                if i not in autos or j not in autos:
                    raise ValueError("the Appendix A map of pair %s needs the auto pairs of both channels"
                                     % ((i, j),))
            if self.s3_max_disp > 0:
                for c in range(self.n_channels):
                    if c not in autos:
                        raise ValueError("the Appendix A map of S3 needs the auto pair of channel %d" % c)
                for l in range(self.n_levels):
                    if 2 * self.s3_P(l) > self.max_disp[l]:
                        raise ValueError("the Appendix A map of S3 reads S2(r_a - r_b): needs 2 P3 <= P")

    @property
    def ndim(self):
        return len(self.shape)

    def level_shape(self, l: int) -> Tuple[int, ...]:
        return tuple(s >> l for s in self.shape)

    def disp(self, l: int, pair) -> np.ndarray:
        P = self.max_disp[l]
        return half_box(self.ndim, P) if pair[0] == pair[1] else box(self.ndim, P)

    def s3_P(self, l: int) -> int:
        return min(self.s3_max_disp, self.max_disp[l])

    def s3_vecs(self, l: int) -> np.ndarray:
        """The M displacements of the three-point block of level l (full box, lexicographic)."""
        return box(self.ndim, self.s3_P(l))

    def s3_index_pairs(self, l: int):
        """(ia, ib) with ia <= ib, ia-major: the unordered vector pairs (S3 is symmetric)."""
        M = len(self.s3_vecs(l))
        return np.triu_indices(M)

    def blocks(self):
        """Every block in descriptor order: ('s2', level, pair, offset, count) for the
        pairs, then ('s3', level, channel, offset, count) for the three-point blocks."""
        out, off = [], 0
        for l in range(self.n_levels):
            for p in self.pairs:
                k = len(self.disp(l, p))
                out.append(("s2", l, p, off, k))
                off += k
            if self.s3_max_disp > 0:
                M = len(self.s3_vecs(l))
                for c in range(self.n_channels):
                    k = M * (M + 1) // 2
                    out.append(("s3", l, c, off, k))
                    off += k
        return out

    def layout(self):
        """List of (level, pair, offset, count) of the two-point blocks, in descriptor order."""
        return [(l, p, off, k) for (kind, l, p, off, k) in self.blocks() if kind == "s2"]

    def s3_layout(self):
        """List of (level, channel, offset, count) of the three-point blocks."""
        return [(l, c, off, k) for (kind, l, c, off, k) in self.blocks() if kind == "s3"]

    @property
    def K(self) -> int:
        return sum(e[4] for e in self.blocks())


# ----------------------------------------------------------------------------
# multigrid pyramid (Sec. 3.3)
# ----------------------------------------------------------------------------
def pool(f: np.ndarray) -> np.ndarray:
    """Mean over each 2^d block of a [C][n...] field (one level coarser)."""
    C = f.shape[0]
    sh = f.shape[1:]
    d = len(sh)
    newshape = [C]
    for s in sh:
        newshape += [s // 2, 2]
    g = f.reshape(newshape)
    return g.mean(axis=tuple(2 + 2 * a for a in range(d)))


def pool_adjoint(g: np.ndarray) -> np.ndarray:
    """Transpose of pool: each coarse value spreads 2^-d of itself to its children."""
    d = g.ndim - 1
    out = g
    for a in range(d):
        out = np.repeat(out, 2, axis=1 + a)
    return out / float(2 ** d)


def pyramid(phi: np.ndarray, n_levels: int) -> List[np.ndarray]:
    levels = [np.asarray(phi, dtype=np.float64)]
    for _ in range(1, n_levels):
        levels.append(pool(levels[-1]))
    return levels


# ----------------------------------------------------------------------------
# descriptor, error, gradient
# ----------------------------------------------------------------------------
def _pair_corr(a, b, r, spec: Spec):
    """One (level, pair) block before any Appendix A map: S2 or Sbar."""
    if spec.descriptor == "s2":
        return _native.corr(a, b, r)
    return _native.sbar(a, b, r, spec.alpha, soft_threshold_constants(spec.alpha))


def descriptor(phi: np.ndarray, spec: Spec) -> np.ndarray:
    """Descriptor of one field phi[C][n...], every level and pair in order:
    s2:     S_ij^(l)(r) = (1/N_l) sum_x phi_i(x) phi_j(x + r);
    sbar:   (1/N_l) sum_x f((phi_i(x) + phi_j(x + r)) / 2)^2;
    stilde: sbar mapped back by Appendix A (correct_sbar)."""
    lv = pyramid(phi, spec.n_levels)
    out = np.zeros(spec.K, np.float64)
    for (l, (i, j), off, k) in spec.layout():
        out[off:off + k] = _pair_corr(lv[l][i], lv[l][j], spec.disp(l, (i, j)), spec)
    for (l, c, off, k) in spec.s3_layout():
        ia, ib = spec.s3_index_pairs(l)
        out[off:off + k] = _native.s3(lv[l][c], spec.s3_vecs(l), ia, ib, *_s3_mode(spec))
    if spec.descriptor == "stilde":
        out = correct_sbar(out, spec)
        out = correct_s3(out, spec)
    return out


def _s3_mode(spec: Spec):
    """(mode, alpha, (c1, c2, c3)) of the three-point blocks: the product form with the
    S2 descriptor, the soft-threshold realisations otherwise."""
    if spec.descriptor == "s2":
        return 0, 0.0, (0.0, 0.0, 0.0)
    return 1, spec.alpha, soft_threshold_constants(spec.alpha)


def _s2_index(spec: Spec, l: int, c: int, r) -> int:
    """Descriptor index of S2_cc(r) at level l for any r with |r_i| <= P_l (point
    symmetry maps r outside the half box to -r)."""
    r = tuple(int(v) for v in r)
    if not in_half(r):
        r = tuple(-v for v in r)
    (_, _, off, _) = [e for e in spec.layout() if e[0] == l and e[1] == (c, c)][0]
    hb = half_box(spec.ndim, spec.max_disp[l])
    return off + int(np.flatnonzero((hb == np.array(r)).all(axis=1))[0])


def _s3_map_terms(spec: Spec, l: int, c: int):
    """For each entry k of the (l, c) three-point block: a list of (coefficient, index)
    such that S3~_k = coef_bar * Sbar3_k + sum coefficient * S2~[index], following
    Appendix A eq. (s3rfroms3rbar) with h = f(1/2):
      r_a = r_b, or one of them 0:  S2~ of the other (coef_bar = 0);
      otherwise: (Sbar3 - h (S2(r_a) + S2(r_b)) - h^2 (S2(0) - S2(r_a) - S2(r_b) + S2(r_a - r_b))) / (1 - 2h)."""
    h = float(soft_threshold(0.5, spec.alpha))
    vecs = spec.s3_vecs(l)
    ia, ib = spec.s3_index_pairs(l)
    out = []
    for a_i, b_i in zip(ia, ib):
        a, b = vecs[a_i], vecs[b_i]
        if a_i == b_i or not b.any():
            out.append((0.0, [(1.0, _s2_index(spec, l, c, a))]))
        elif not a.any():
            out.append((0.0, [(1.0, _s2_index(spec, l, c, b))]))
        else:
            q = 1.0 / (1.0 - 2.0 * h)
            out.append((q, [((-h + h * h) * q, _s2_index(spec, l, c, a)),
                            ((-h + h * h) * q, _s2_index(spec, l, c, b)),
                            (-h * h * q, _s2_index(spec, l, c, np.zeros_like(a))),
                            (-h * h * q, _s2_index(spec, l, c, a - b))]))
    return out


def correct_s3(S: np.ndarray, spec: Spec) -> np.ndarray:
    """Appendix A eq. (s3rfroms3rbar) on every three-point block; S holds the corrected
    two-point blocks (correct_sbar) and the raw Sbar3 blocks."""
    out = np.array(S, np.float64, copy=True)
    for (l, c, off, k) in spec.s3_layout():
        for e, (cb, terms) in enumerate(_s3_map_terms(spec, l, c)):
            out[off + e] = cb * S[off + e] + sum(w * S[i] for (w, i) in terms)
    return out


def correct_s3_adjoint(G: np.ndarray, spec: Spec) -> np.ndarray:
    """Transpose of correct_s3 (linear in S): the three-point cotangent scales by the
    Sbar3 coefficient, and each S2~ entry a map reads collects coefficient x cotangent."""
    G = np.asarray(G, np.float64)
    out = np.array(G, copy=True)
    for (l, c, off, k) in spec.s3_layout():
        for e, (cb, terms) in enumerate(_s3_map_terms(spec, l, c)):
            out[off + e] = cb * G[off + e]
            for (w, i) in terms:
                out[i] += w * G[off + e]
    return out


def _f_half_sq(spec: Spec) -> float:
    return float(soft_threshold(0.5, spec.alpha)) ** 2


def _level_vf(S: np.ndarray, spec: Spec, l: int):
    """Sbar_cc(0) of every channel c at level l (r = 0 is the first entry of a half box)."""
    return {i: S[off] for (ll, (i, j), off, k) in spec.layout() if ll == l and i == j}


def correct_sbar(Sbar: np.ndarray, spec: Spec) -> np.ndarray:
    """Appendix A, eq. (s2rfroms2rbar), per level and pair, with F = f(1/2)^2:
    S(r) = (Sbar(r) - F (Sbar_ii(0) + Sbar_jj(0))) / (1 - 2F).  For an auto pair
    at r != 0 this is the paper's map; at r = 0 it returns Sbar(0)."""
    F = _f_half_sq(spec)
    out = np.array(Sbar, np.float64, copy=True)
    for l in range(spec.n_levels):
        vf = _level_vf(Sbar, spec, l)
        for (ll, (i, j), off, k) in spec.layout():
            if ll == l:
                out[off:off + k] = (Sbar[off:off + k] - F * (vf[i] + vf[j])) / (1.0 - 2.0 * F)
    return out


def correct_sbar_adjoint(G: np.ndarray, spec: Spec) -> np.ndarray:
    """Transpose of correct_sbar (it is linear in Sbar): every two-point entry is
    scaled by 1/(1 - 2F), and each channel's r = 0 auto entry also collects
    -F/(1 - 2F) times the cotangent of every entry whose map reads it; three-point
    entries pass through unchanged."""
    F = _f_half_sq(spec)
    G = np.asarray(G, np.float64)
    out = np.array(G, copy=True)
    for (_, _, off, k) in spec.layout():
        out[off:off + k] = G[off:off + k] / (1.0 - 2.0 * F)
    for l in range(spec.n_levels):
        lay = [e for e in spec.layout() if e[0] == l]
        auto_off = {i: off for (_, (i, j), off, k) in lay if i == j}
        for (_, (i, j), off, k) in lay:
            t = float(np.sum(G[off:off + k]))
            out[auto_off[i]] -= F / (1.0 - 2.0 * F) * t
            out[auto_off[j]] -= F / (1.0 - 2.0 * F) * t
    return out


def level_weights_per_entry(spec: Spec) -> np.ndarray:
    w = np.zeros(spec.K, np.float64)
    for (_, l, _, off, k) in spec.blocks():
        w[off:off + k] = spec.level_weight[l]
    return w


def error_Z(spec: Spec) -> float:
    """Z = sum_l w_l^2 K_l (entries of all pairs at level l)."""
    w = level_weights_per_entry(spec)
    return float(np.sum(w * w))


def loss(S: np.ndarray, S_des: np.ndarray, spec: Spec):
    """E = (1/Z) sum w_l^2 (S - S_des)^2 and its cotangent G = dE/dS."""
    w2 = level_weights_per_entry(spec) ** 2
    Z = float(np.sum(w2))
    diff = np.asarray(S, np.float64) - np.asarray(S_des, np.float64)
    E = float(np.sum(w2 * diff * diff) / Z)
    G = 2.0 * w2 * diff / Z
    return E, G


def _pair_adjoint(a, b, r, G, spec: Spec):
    if spec.descriptor == "s2":
        return _native.corr_adjoint(a, b, r, G)
    return _native.sbar_adjoint(a, b, r, spec.alpha, soft_threshold_constants(spec.alpha), G)


def adjoint(phi: np.ndarray, G: np.ndarray, spec: Spec) -> np.ndarray:
    """d/dphi of sum_k G[k] S[k] (all levels, all pairs), shape of phi."""
    if spec.descriptor == "stilde":
        G = correct_sbar_adjoint(correct_s3_adjoint(G, spec), spec)
    lv = pyramid(phi, spec.n_levels)
    grads = [np.zeros_like(f) for f in lv]
    for (l, (i, j), off, k) in spec.layout():
        ga, gb = _pair_adjoint(lv[l][i], lv[l][j], spec.disp(l, (i, j)), G[off:off + k], spec)
        grads[l][i] += ga
        grads[l][j] += gb
    for (l, c, off, k) in spec.s3_layout():
        ia, ib = spec.s3_index_pairs(l)
        mode, alpha, cc = _s3_mode(spec)
        grads[l][c] += _native.s3_adjoint(lv[l][c], spec.s3_vecs(l), ia, ib, mode, G[off:off + k], alpha, cc)
    acc = grads[-1]
    for l in range(spec.n_levels - 2, -1, -1):
        acc = grads[l] + pool_adjoint(acc)
    return acc


def loss_grad(phi: np.ndarray, S_des: np.ndarray, spec: Spec):
    S = descriptor(phi, spec)
    E, G = loss(S, S_des, spec)
    return E, adjoint(phi, G, spec), S


def descriptor_at(phi: np.ndarray, spec: Spec, level: int, pair, r: np.ndarray) -> np.ndarray:
    """S2 or Sbar (no Appendix A map) at a list of displacements of one (level, pair)."""
    lv = pyramid(phi, level + 1)
    return _pair_corr(lv[level][pair[0]], lv[level][pair[1]], np.asarray(r), spec)


def adjoint_at_single_level(phi: np.ndarray, G: np.ndarray, spec: Spec, vox: np.ndarray) -> np.ndarray:
    """Gradient at listed finest-level voxels for a single-level spec: [C][nv]."""
    if spec.n_levels != 1 or spec.s3_max_disp > 0:
        raise ValueError("sampled adjoint is defined here for one level of two-point blocks only")
    if spec.descriptor == "stilde":
        G = correct_sbar_adjoint(G, spec)
    out = np.zeros((spec.n_channels, len(vox)), np.float64)
    for (l, (i, j), off, k) in spec.layout():
        if spec.descriptor == "s2":
            ga, gb = _native.corr_adjoint_at(phi[i], phi[j], spec.disp(l, (i, j)), G[off:off + k], vox)
        else:
            ga, gb = _native.sbar_adjoint_at(phi[i], phi[j], spec.disp(l, (i, j)), spec.alpha,
                                             soft_threshold_constants(spec.alpha), G[off:off + k], vox)
        out[i] += ga
        out[j] += gb
    return out


# ----------------------------------------------------------------------------
# box penalty (Sec. 3.1): E^bc = sum [ (M-1)H(M-1)/N + (-M)H(-M)/N ]^2, H(0) = 0
# ----------------------------------------------------------------------------
def penalty(phi: np.ndarray, lo: float = 0.0, hi: float = 1.0):
    """E^bc and its gradient for every explicit channel; N = voxels per channel."""
    phi = np.asarray(phi, np.float64)
    N = float(np.prod(phi.shape[1:]))
    over = np.where(phi - hi > 0, phi - hi, 0.0)
    under = np.where(lo - phi > 0, lo - phi, 0.0)
    t = over / N + under / N
    Ebc = float(np.sum(t * t))
    dt = np.where(phi - hi > 0, 1.0 / N, 0.0) - np.where(lo - phi > 0, 1.0 / N, 0.0)
    return Ebc, 2.0 * t * dt


def penalised_loss_grad(phi, S_des, spec, kappa=1.0, lo=0.0, hi=1.0):
    """L = E + lambda E^bc of Sec. 3.1 (eq. L_func_dMCR) with lambda = kappa * E
    (lambda proportional to E; the constant is not given) held constant in the
    gradient: returns (L, dE/dphi + lambda dE^bc/dphi, E)."""
    E, g, S = loss_grad(phi, S_des, spec)
    Ebc, gbc = penalty(phi, lo, hi)
    lam = kappa * E
    return E + lam * Ebc, g + lam * gbc, E


# ----------------------------------------------------------------------------
# optimiser references
# ----------------------------------------------------------------------------
def lbfgs_direction(g: np.ndarray, s_hist: Sequence[np.ndarray], y_hist: Sequence[np.ndarray], gamma=None):
    """Two-loop recursion (Nocedal & Wright, Alg. 7.4), FP64: returns -H g.

    s_hist / y_hist are ordered oldest first.  Initial scaling gamma as given, else
    s'y / y'y of the newest pair (identity if the history is empty)."""
    q = np.array(g, np.float64, copy=True).reshape(-1)
    m = len(s_hist)
    alpha = np.zeros(m)
    rho = np.zeros(m)
    for i in range(m - 1, -1, -1):
        s, y = s_hist[i].reshape(-1), y_hist[i].reshape(-1)
        rho[i] = 1.0 / float(np.dot(y, s))
        alpha[i] = rho[i] * float(np.dot(s, q))
        q -= alpha[i] * y
    if gamma is not None:
        q *= gamma
    elif m:
        s, y = s_hist[-1].reshape(-1), y_hist[-1].reshape(-1)
        q *= float(np.dot(s, y)) / float(np.dot(y, y))
    for i in range(m):
        s, y = s_hist[i].reshape(-1), y_hist[i].reshape(-1)
        beta = rho[i] * float(np.dot(y, q))
        q += (alpha[i] - beta) * s
    return -q.reshape(np.shape(g))


def reconstruct_lbfgs_projected(S_des, spec: Spec, phi0, iters, m=10, c1=1e-4, max_ls=20, lo=0.0, hi=1.0,
                                bounds="project", kappa=1.0):
    """L-BFGS on the relaxed problem of Sec. 3 (eqs. dMCR-Min_Prob, L_func_dMCR), FP64,
    with the same rules as the GPU driver; returns (phi, [f after each iteration],
    [evaluations of each iteration]).

    bounds="project" keeps lo <= phi <= hi by projection; bounds="penalty" leaves
    phi free and minimises L = E + lambda E^bc (E^bc as printed in Sec. 3.1,
    lambda = kappa E of the current point, held constant in the gradient and in
    the line search that starts there; f is then L with the point's own lambda).

    Each iteration: d = -H g by the two-loop recursion over the valid pairs among
    the last m iterations' pairs, initial scaling gamma = s'y / y'y of the newest
    valid pair (1 after a reset); with projection, components of d that push an
    active bound outward are zeroed; if g'd >= 0 the history is cleared and d = -g
    (projected).  Backtracking along the (projected) path x_t = clip(x + a d),
    halving a, with the Armijo test f_x(x_t) <= f(x) + c1 g'(x_t - x) (Nocedal &
    Wright, Alg. 3.1 on the projected path; f_x uses the lambda of x); the first
    trial is a = 1/|g| while no step has been accepted since the last reset, else 1.
    An accepted step records the pair s = x_t - x, y = g_t - g, valid if
    s'y > eps y'y and y'y > 0; a failed search records no pair and clears the
    history."""
    penal = bounds == "penalty"
    clip = (lambda v: v) if penal else (lambda v: np.clip(v, lo, hi))

    def evaluate(v):
        """(E, E^bc, gradient with lambda = kappa E(v))"""
        if penal:
            L, g_, E_ = penalised_loss_grad(v, S_des, spec, kappa, lo, hi)
            return E_, penalty(v, lo, hi)[0], g_
        E_, g_, _ = loss_grad(v, S_des, spec)
        return E_, 0.0, g_

    x = clip(np.asarray(phi0, np.float64))
    E, Ebc, g = evaluate(x)
    f = E + kappa * E * Ebc
    ring = []           # pairs of the last m iterations, None where none was recorded
    gamma, hist = 1.0, 0
    Es, evals = [], []
    eps = np.finfo(np.float64).eps

    def project_dir(d_):
        if not penal:
            d_[((x <= lo) & (d_ < 0)) | ((x >= hi) & (d_ > 0))] = 0.0
        return d_

    for _ in range(iters):
        valid = [p for p in ring if p is not None]
        d = project_dir(lbfgs_direction(g, [p[0] for p in valid], [p[1] for p in valid], gamma=gamma))
        if not float(np.sum(g * d)) < 0.0:
            ring = [None] * len(ring)
            gamma, hist = 1.0, 0
            d = project_dir(-g.copy())
        gn = float(np.sqrt(np.sum(g * g)))
        a = 1.0 / gn if (hist == 0 and gn > 0.0) else 1.0
        lam = kappa * E
        accepted, n_ev = False, 0
        for _ls in range(max_ls):
            xt = clip(x + a * d)
            Et, Ebct, gt = evaluate(xt)
            n_ev += 1
            dd = float(np.sum(g * (xt - x)))
            ft_x = Et + lam * Ebct
            if np.isfinite(ft_x) and dd < 0.0 and ft_x <= f + c1 * dd:
                accepted = True
                break
            a *= 0.5
        pair = None
        if accepted:
            s_, y_ = xt - x, gt - g
            sy, yy = float(np.sum(s_ * y_)), float(np.sum(y_ * y_))
            if sy > eps * yy and yy > 0.0:
                pair = (s_, y_)
                gamma = sy / yy
            x, g, E = xt, gt, Et
            f = Et + kappa * Et * Ebct
            hist = min(hist + 1, m)
        ring = (ring + [pair])[-m:]
        if not accepted:
            ring = [None] * len(ring)
            gamma, hist = 1.0, 0
        Es.append(f)
        evals.append(n_ev)
    return x, Es, evals


def adam_step(x, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-7, lo=None, hi=None):
    """One Adam update (Kingma & Ba, Alg. 1; the paper's optimizer, Appendix B) in FP64:
    biased moments m, v, their bias corrections at step t >= 1, the step
    lr * m_hat / (sqrt(v_hat) + eps), then projection onto [lo, hi] if given.
    Returns (x, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    x = x - lr * m_hat / (np.sqrt(v_hat) + eps)
    if lo is not None:
        x = np.clip(x, lo, hi)
    return x, m, v


def reconstruct_adam(S_des, spec: Spec, phi0, iters, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-7,
                     lo=0.0, hi=1.0, tol=0.0):
    """Projected Adam on the oracle's (E, dE/dphi): start from clip(phi0), take up to
    `iters` steps, stop once E <= tol.  Returns (phi, E_final, steps taken)."""
    x = np.clip(np.asarray(phi0, np.float64), lo, hi)
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    E, g, _ = loss_grad(x, S_des, spec)
    t = 0
    while t < iters and E > tol:
        t += 1
        x, m, v = adam_step(x, g, m, v, t, lr, beta1, beta2, eps, lo, hi)
        E, g, _ = loss_grad(x, S_des, spec)
    return x, float(E), t


def level_spec(spec: Spec, l: int) -> Spec:
    """The single-level spec of level l (its grid, P_l, the same pairs and kinds)."""
    return Spec(shape=spec.level_shape(l), n_channels=spec.n_channels, n_levels=1,
                max_disp=(spec.max_disp[l],), level_weight=(1.0,), pairs=spec.pairs,
                descriptor=spec.descriptor, alpha=spec.alpha, s3_max_disp=spec.s3_max_disp)


def level_slice(spec: Spec, l: int) -> slice:
    """Entries of level l in the multigrid descriptor (level-major order)."""
    offs = [off for (_, ll, _, off, _) in spec.blocks() if ll == l]
    ends = [off + k for (_, ll, _, off, k) in spec.blocks() if ll == l]
    return slice(min(offs), max(ends))


def upsample(g: np.ndarray) -> np.ndarray:
    """Nearest-neighbour upsampling of a [C][n...] field by 2 along every axis."""
    out = g
    for a in range(g.ndim - 1):
        out = np.repeat(out, 2, axis=1 + a)
    return out


def reconstruct_coarse_to_fine(S_des, spec: Spec, phi0, maxiter=100, maxcor=10, lo=0.0, hi=1.0):
    """Sequential coarse-to-fine reference: the start field pooled to the coarsest
    level, each level reconstructed alone (SciPy L-BFGS-B on its single-level loss
    against its slice of the target), the result upsampled to start the next finer
    level.  Returns (phi, multigrid E of the result)."""
    lv = pyramid(np.asarray(phi0, np.float64), spec.n_levels)
    x = lv[-1]
    for l in range(spec.n_levels - 1, -1, -1):
        if l < spec.n_levels - 1:
            x = upsample(x)
        ls = level_spec(spec, l)
        x, _, _, _ = reconstruct_lbfgsb(np.asarray(S_des)[level_slice(spec, l)], ls, x, maxiter, maxcor, lo, hi)
    E = loss(descriptor(x, spec), S_des, spec)[0]
    return x, float(E)


def reconstruct_lbfgsb(S_des, spec: Spec, phi0, maxiter=100, maxcor=10, lo=0.0, hi=1.0):
    """Reference reconstruction: SciPy L-BFGS-B on the oracle's (E, dE/dphi) in FP64,
    bounds [lo, hi] on every voxel.  Returns (phi, E_final, n_iter, n_eval)."""
    from scipy.optimize import minimize

    shape = np.shape(phi0)
    counter = {"n": 0}

    def fun(x):
        counter["n"] += 1
        E, g, _ = loss_grad(x.reshape(shape), S_des, spec)
        return E, g.reshape(-1)

    res = minimize(fun, np.asarray(phi0, np.float64).reshape(-1), jac=True, method="L-BFGS-B",
                   bounds=[(lo, hi)] * int(np.prod(shape)),
                   options={"maxiter": maxiter, "maxcor": maxcor, "ftol": 0.0, "gtol": 0.0})
    return res.x.reshape(shape), float(res.fun), int(res.nit), counter["n"]
