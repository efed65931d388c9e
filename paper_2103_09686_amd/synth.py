"""Seeded synthetic microstructures (inputs only; none of the descriptor's arithmetic).

These generators stand in for the paper's pyMKS and literature micrographs
(Sec. 5.2), which are not available: periodic Boolean models of overlapping
disks / spheres, thresholded periodic Gaussian random fields, a three-phase
mix of spheres and randomly oriented ellipsoids, checkerboards and uniform
noise.  Every function takes an explicit seed and returns float64 arrays of
phase indicators, shape [C][n...] with C = number of phases - 1 (the matrix
phase is implicit).  Both the oracle tests and the GPU tests draw their
inputs from here.
"""
import numpy as np


def uniform(shape, seed, channels=1):
    """i.i.d. U(0,1) soft field [channels][shape]."""
    rng = np.random.default_rng(seed)
    return rng.random((channels,) + tuple(shape))


def _stamp_offsets(radius, ndim):
    r = int(np.ceil(radius))
    ax = np.arange(-r, r + 1)
    grid = np.stack(np.meshgrid(*([ax] * ndim), indexing="ij"), axis=-1).reshape(-1, ndim)
    return grid


def _fill_until(mask, target_vf, propose, rng, allowed=None, max_objects=10_000_000):
    """Add objects (boolean stamps from propose(rng)) until the covered fraction of
    `mask` reaches target_vf.  Only voxels where `allowed` is True may be claimed."""
    N = mask.size
    shape = np.array(mask.shape)
    count = 0
    flat = mask.reshape(-1)
    strides = np.array([int(np.prod(shape[a + 1:])) for a in range(len(shape))])
    covered = int(np.count_nonzero(flat))
    while covered < target_vf * N and count < max_objects:
        centre, offsets = propose(rng)
        idx = np.mod(offsets + centre[None, :], shape[None, :])
        lin = np.unique(idx @ strides)
        if allowed is not None:
            lin = lin[allowed.reshape(-1)[lin]]
        covered += int(np.count_nonzero(~flat[lin]))
        flat[lin] = True
        count += 1
    return count


def boolean_spheres(shape, radius, vf, seed):
    """Overlapping periodic disks (2-D) or spheres (3-D) of the given radius, centres
    uniform on the grid, added until the covered fraction reaches vf.  Returns
    ([1][shape] indicator, actual volume fraction)."""
    shape = tuple(shape)
    nd = len(shape)
    rng = np.random.default_rng(seed)
    offs = _stamp_offsets(radius, nd)
    offs = offs[np.sum(offs.astype(np.float64) ** 2, axis=1) <= radius * radius + 1e-9]
    mask = np.zeros(shape, dtype=bool)

    def propose(rng):
        c = np.array([rng.integers(0, s) for s in shape])
        return c, offs

    _fill_until(mask, vf, propose, rng)
    return mask[None].astype(np.float64), float(mask.mean())


def _random_rotation(rng, nd):
    """Uniformly random rotation matrix (QR of a Gaussian matrix, sign-fixed)."""
    A = rng.standard_normal((nd, nd))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def _ellipsoid_offsets(semi, rot):
    nd = len(semi)
    r = int(np.ceil(max(semi)))
    ax = np.arange(-r, r + 1)
    grid = np.stack(np.meshgrid(*([ax] * nd), indexing="ij"), axis=-1).reshape(-1, nd)
    local = grid.astype(np.float64) @ rot  # coordinates in the body frame
    inside = np.sum((local / np.asarray(semi, np.float64)[None, :]) ** 2, axis=1) <= 1.0
    return grid[inside]


def spheres_and_ellipsoids(shape, sphere_radius=6, vf1=0.20, semi_axes=(10, 4, 4), vf2=0.15, seed=0):
    """Three-phase medium: phase 1 = overlapping spheres (disks in 2-D) up to vf1,
    then phase 2 = randomly oriented ellipsoids (ellipses) that claim only matrix
    voxels, up to vf2.  Returns ([2][shape] indicators, (vf1, vf2) actual)."""
    shape = tuple(shape)
    nd = len(shape)
    semi = tuple(semi_axes[:nd])
    rng = np.random.default_rng(seed)
    p1, _ = boolean_spheres(shape, sphere_radius, vf1, int(rng.integers(1 << 31)))
    m1 = p1[0] > 0.5
    m2 = np.zeros(shape, dtype=bool)

    def propose(rng):
        c = np.array([rng.integers(0, s) for s in shape])
        return c, _ellipsoid_offsets(semi, _random_rotation(rng, nd))

    allowed = ~m1
    _fill_until(m2, vf2, propose, rng, allowed=allowed)
    return np.stack([m1, m2]).astype(np.float64), (float(m1.mean()), float(m2.mean()))


def gaussian_random_field(shape, corr_len, seed):
    """Periodic stationary Gaussian field with covariance exp(-|r|^2 / (2 l^2)),
    unit variance, by spectral filtering of white noise."""
    shape = tuple(shape)
    rng = np.random.default_rng(seed)
    # periodic minimum-image squared distance from the origin
    d2 = np.zeros(shape)
    for a, n in enumerate(shape):
        k = np.arange(n)
        k = np.minimum(k, n - k).astype(np.float64)
        sl = [1] * len(shape)
        sl[a] = n
        d2 = d2 + (k ** 2).reshape(sl)
    cov = np.exp(-d2 / (2.0 * corr_len ** 2))
    spec = np.clip(np.real(np.fft.fftn(cov)), 0.0, None)
    w = rng.standard_normal(shape)
    f = np.real(np.fft.ifftn(np.fft.fftn(w) * np.sqrt(spec)))
    return (f - f.mean()) / f.std()


def threshold_top(field, vf):
    """Indicator of the round(vf*N) largest values (exact volume fraction)."""
    flat = field.reshape(-1)
    k = int(round(vf * flat.size))
    out = np.zeros(flat.size, dtype=np.float64)
    if k > 0:
        idx = np.argpartition(-flat, k - 1)[:k]
        out[idx] = 1.0
    return out.reshape(field.shape)


def grf_two_phase(shape, corr_len, vf, seed):
    """Thresholded periodic GRF: phase 1 = the top vf fraction.  [1][shape]."""
    return threshold_top(gaussian_random_field(shape, corr_len, seed), vf)[None]


def grf_three_phase(shape, corr_len, vf1, vf2, seed):
    """Two thresholds of one periodic GRF: phase 1 = top vf1, phase 2 = the next vf2."""
    f = gaussian_random_field(shape, corr_len, seed)
    a = threshold_top(f, vf1)
    b = threshold_top(f, vf1 + vf2) - a
    return np.stack([a, b])


def checkerboard(shape, square):
    """Periodic checkerboard with squares (cubes) of side `square` pixels.  [1][shape]."""
    idx = np.indices(tuple(shape)).sum(axis=0) if square == 1 else \
        sum((np.indices(tuple(shape))[a] // square) for a in range(len(shape)))
    return (idx % 2 == 0).astype(np.float64)[None]
