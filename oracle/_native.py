"""Loader for the oracle's C core (oracle.c).

TEST INFRASTRUCTURE ONLY: the oracle is imported by the test suite, the smoke
check and the CPU-baseline leg of the benchmark, never by the product path.
The C core is compiled with gcc (no fast-math, so every FP64 sum is evaluated
in the order the source writes it).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force=False):
    """Compile oracle.c into liboracle.so (gcc, -O2 -fopenmp, FP64 as written)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.ora_corr.argtypes = [ctypes.c_int] * 3 + [_dp, _dp, ctypes.c_int, _ip, _dp]
        L.ora_corr.restype = None
        L.ora_corr_adjoint.argtypes = [ctypes.c_int] * 3 + [_dp, _dp, ctypes.c_int, _ip, _dp, _dp, _dp]
        L.ora_corr_adjoint.restype = None
        L.ora_corr_adjoint_at.argtypes = ([ctypes.c_int] * 3 + [_dp, _dp, ctypes.c_int, _ip, _dp,
                                          ctypes.c_int, _ip, _dp, _dp])
        L.ora_corr_adjoint_at.restype = None
        L.ora_sbar.argtypes = [ctypes.c_int] * 3 + [_dp, _dp, ctypes.c_int, _ip, _dp, _dp]
        L.ora_sbar.restype = None
        L.ora_sbar_adjoint.argtypes = [ctypes.c_int] * 3 + [_dp, _dp, ctypes.c_int, _ip, _dp, _dp, _dp, _dp]
        L.ora_sbar_adjoint.restype = None
        L.ora_sbar_adjoint_at.argtypes = ([ctypes.c_int] * 3 + [_dp, _dp, ctypes.c_int, _ip, _dp, _dp,
                                          ctypes.c_int, _ip, _dp, _dp])
        L.ora_sbar_adjoint_at.restype = None
        L.ora_s3.argtypes = [ctypes.c_int] * 3 + [_dp, _ip, ctypes.c_int, _ip, _ip, ctypes.c_int, _dp, _dp]
        L.ora_s3.restype = None
        L.ora_s3_adjoint.argtypes = ([ctypes.c_int] * 3 + [_dp, _ip, ctypes.c_int, _ip, _ip, ctypes.c_int, _dp,
                                     _dp, _dp])
        L.ora_s3_adjoint.restype = None
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _d(x):
    return x.ctypes.data_as(_dp)


def _i(x):
    return x.ctypes.data_as(_ip)


def _as3(field):
    """View a 2-D or 3-D field as n0 x n1 x n2 (2-D: n0 = 1)."""
    f = np.ascontiguousarray(field, dtype=np.float64)
    if f.ndim == 2:
        f = f.reshape((1,) + f.shape)
    if f.ndim != 3:
        raise ValueError("field must be 2-D or 3-D")
    return f


def _r3(r, ndim):
    r = np.asarray(r, dtype=np.int32).reshape(-1, ndim)
    if ndim == 2:
        r = np.concatenate([np.zeros((r.shape[0], 1), np.int32), r], axis=1)
    return np.ascontiguousarray(r, dtype=np.int32)


def corr(a, b, r):
    """S[k] = (1/N) sum_x a(x) b(x + r_k), periodic, FP64."""
    ndim = np.ndim(a)
    A, B = _as3(a), _as3(b)
    R = _r3(r, ndim)
    S = np.zeros(R.shape[0], np.float64)
    lib().ora_corr(A.shape[0], A.shape[1], A.shape[2], _d(A), _d(B), R.shape[0], _i(R), _d(S))
    return S


def corr_adjoint(a, b, r, G):
    """(ga, gb): gradients of sum_k G[k] S_ab(r_k) w.r.t. a and b (separately)."""
    ndim = np.ndim(a)
    A, B = _as3(a), _as3(b)
    R = _r3(r, ndim)
    Gk = np.ascontiguousarray(G, dtype=np.float64)
    ga = np.zeros_like(A)
    gb = np.zeros_like(B)
    lib().ora_corr_adjoint(A.shape[0], A.shape[1], A.shape[2], _d(A), _d(B), R.shape[0], _i(R),
                           _d(Gk), _d(ga), _d(gb))
    return ga.reshape(np.shape(a)), gb.reshape(np.shape(b))


def corr_adjoint_at(a, b, r, G, vox):
    """Adjoint evaluated only at the listed voxels (rows of vox, ndim columns)."""
    ndim = np.ndim(a)
    A, B = _as3(a), _as3(b)
    R = _r3(r, ndim)
    V = _r3(vox, ndim)
    Gk = np.ascontiguousarray(G, dtype=np.float64)
    ga = np.zeros(V.shape[0], np.float64)
    gb = np.zeros(V.shape[0], np.float64)
    lib().ora_corr_adjoint_at(A.shape[0], A.shape[1], A.shape[2], _d(A), _d(B), R.shape[0], _i(R),
                              _d(Gk), V.shape[0], _i(V), _d(ga), _d(gb))
    return ga, gb


def _coef(alpha, c):
    return np.ascontiguousarray([alpha, c[0], c[1], c[2]], dtype=np.float64)


def sbar(a, b, r, alpha, c):
    """Sbar[k] = (1/N) sum_x f((a(x) + b(x + r_k)) / 2)^2 with the logistic soft
    threshold f of slope alpha and constants c = (c1, c2, c3), periodic, FP64."""
    ndim = np.ndim(a)
    A, B = _as3(a), _as3(b)
    R = _r3(r, ndim)
    S = np.zeros(R.shape[0], np.float64)
    co = _coef(alpha, c)
    lib().ora_sbar(A.shape[0], A.shape[1], A.shape[2], _d(A), _d(B), R.shape[0], _i(R), _d(co), _d(S))
    return S


def sbar_adjoint(a, b, r, alpha, c, G):
    """(ga, gb): gradients of sum_k G[k] Sbar_ab(r_k) w.r.t. a and b (separately)."""
    ndim = np.ndim(a)
    A, B = _as3(a), _as3(b)
    R = _r3(r, ndim)
    Gk = np.ascontiguousarray(G, dtype=np.float64)
    co = _coef(alpha, c)
    ga = np.zeros_like(A)
    gb = np.zeros_like(B)
    lib().ora_sbar_adjoint(A.shape[0], A.shape[1], A.shape[2], _d(A), _d(B), R.shape[0], _i(R),
                           _d(co), _d(Gk), _d(ga), _d(gb))
    return ga.reshape(np.shape(a)), gb.reshape(np.shape(b))


def sbar_adjoint_at(a, b, r, alpha, c, G, vox):
    """Soft-threshold adjoint evaluated only at the listed voxels."""
    ndim = np.ndim(a)
    A, B = _as3(a), _as3(b)
    R = _r3(r, ndim)
    V = _r3(vox, ndim)
    Gk = np.ascontiguousarray(G, dtype=np.float64)
    co = _coef(alpha, c)
    ga = np.zeros(V.shape[0], np.float64)
    gb = np.zeros(V.shape[0], np.float64)
    lib().ora_sbar_adjoint_at(A.shape[0], A.shape[1], A.shape[2], _d(A), _d(B), R.shape[0], _i(R),
                              _d(co), _d(Gk), V.shape[0], _i(V), _d(ga), _d(gb))
    return ga, gb


def s3(f, vecs, pa, pb, mode, alpha=10.0, c=(0.0, 0.0, 0.0)):
    """Three-point correlation of one field over index pairs (pa[k], pb[k]) into the
    displacement list vecs: mode 0 product form, mode 1 soft threshold."""
    ndim = np.ndim(f)
    F = _as3(f)
    V = _r3(vecs, ndim)
    A = np.ascontiguousarray(pa, dtype=np.int32)
    Bi = np.ascontiguousarray(pb, dtype=np.int32)
    S = np.zeros(len(A), np.float64)
    co = _coef(alpha, c)
    lib().ora_s3(F.shape[0], F.shape[1], F.shape[2], _d(F), _i(V), len(A), _i(A), _i(Bi), int(mode), _d(co), _d(S))
    return S


def s3_adjoint(f, vecs, pa, pb, mode, G, alpha=10.0, c=(0.0, 0.0, 0.0)):
    """Gradient of sum_k G[k] S3_k with respect to the field."""
    ndim = np.ndim(f)
    F = _as3(f)
    V = _r3(vecs, ndim)
    A = np.ascontiguousarray(pa, dtype=np.int32)
    Bi = np.ascontiguousarray(pb, dtype=np.int32)
    Gk = np.ascontiguousarray(G, dtype=np.float64)
    co = _coef(alpha, c)
    g = np.zeros_like(F)
    lib().ora_s3_adjoint(F.shape[0], F.shape[1], F.shape[2], _d(F), _i(V), len(A), _i(A), _i(Bi), int(mode),
                         _d(co), _d(Gk), _d(g))
    return g.reshape(np.shape(f))


def num_threads():
    return lib().ora_num_threads()


def set_num_threads(t):
    lib().ora_set_num_threads(int(t))
