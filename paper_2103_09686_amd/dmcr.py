"""Python binding of libdmcr (include/dmcr.h): argument marshalling only.

Every step of the descriptor, error, adjoint and reconstruction runs in the
HIP kernels of libdmcr.so; PyTorch provides device memory and the stream.
The library is loaded on first use; if it is missing, or no GPU is present,
the calls raise -- there is no CPU fallback.
"""
import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmcr.so")

PATH_AUTO, PATH_FFT, PATH_DIRECT = 0, 1, 2
DESC_S2, DESC_SBAR, DESC_STILDE = 0, 1, 2
FLAG_RECOMPUTE = 1
FLAG_FUSED_PLANES = 2
BOUNDS_NONE, BOUNDS_PROJECT, BOUNDS_PENALTY = 0, 1, 2
OPT_LBFGS, OPT_ADAM = 0, 1
MAX_LEVELS, MAX_CHANNELS, MAX_PAIRS = 8, 4, 10

STATUS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EUNSUPPORTED", -4: "EDEVICE",
          -5: "ENONFINITE", 1: "NOT_CONVERGED", 2: "RUNNING"}
OK, NOT_CONVERGED, RUNNING, ENONFINITE = 0, 1, 2, -5


class DmcrError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__("%s failed: %s (%d)" % (fn, STATUS.get(code, "?"), code))
        self.code = code


class c_spec(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("shape", ctypes.c_int32 * 3),
                ("n_channels", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("max_disp", ctypes.c_int32 * MAX_LEVELS),
                ("level_weight", ctypes.c_double * MAX_LEVELS),
                ("n_pairs", ctypes.c_int32), ("pairs", ctypes.c_int32 * 32),
                ("path", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("descriptor", ctypes.c_int32), ("s3_max_disp", ctypes.c_int32), ("alpha", ctypes.c_double)]


class c_bounds(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double), ("hi", ctypes.c_double), ("mode", ctypes.c_int32),
                ("kappa", ctypes.c_double)]


class c_opt(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("max_ls", ctypes.c_int32),
                ("tol_derr", ctypes.c_double), ("c1", ctypes.c_double),
                ("method", ctypes.c_int32), ("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double)]


class c_slot(ctypes.Structure):
    _fields_ = [("f", ctypes.c_double), ("E", ctypes.c_double), ("hist", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("evals", ctypes.c_int32), ("status", ctypes.c_int32),
                ("active", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class c_ring(ctypes.Structure):
    _fields_ = [("head", ctypes.c_int32), ("count", ctypes.c_int32)]


class c_result(ctypes.Structure):
    _fields_ = [("final_E", ctypes.c_double), ("final_derr", ctypes.c_double),
                ("iters", ctypes.c_int32), ("evals", ctypes.c_int32), ("why", ctypes.c_int32)]


@dataclass
class Spec:
    """One multigrid descriptor: shape of the finest level, channels, levels (0: the
    library's level rule from max_disp[0]), per-level maximum displacement P_l (the
    library clips it to n_l/2 - 1), level weights (empty or 0: the library's default),
    pairs, path, flags, descriptor kind (DESC_*), soft-threshold slope alpha (0: the
    paper's 10) and the three-point range P3 (0: no three-point blocks)."""
    shape: Tuple[int, ...]
    n_channels: int = 1
    n_levels: int = 1
    max_disp: Tuple[int, ...] = (16,)
    level_weight: Tuple[float, ...] = ()
    pairs: Tuple[Tuple[int, int], ...] = ()
    path: int = PATH_AUTO
    flags: int = 0
    descriptor: int = DESC_S2
    alpha: float = 0.0
    s3_max_disp: int = 0

    def __post_init__(self):
        self.shape = tuple(int(s) for s in self.shape)
        d = len(self.shape)
        if len(self.max_disp) == 1 and self.n_levels > 1:
            self.max_disp = tuple(self.max_disp) * self.n_levels
        self.max_disp = tuple(int(p) for p in self.max_disp)
        self.level_weight = tuple(float(w) for w in self.level_weight)
        if not self.pairs:
            self.pairs = tuple((i, j) for i in range(self.n_channels) for j in range(i, self.n_channels))

    @property
    def ndim(self):
        return len(self.shape)

    def c(self) -> c_spec:
        s = c_spec()
        s.ndim = self.ndim
        for a, n in enumerate(self.shape):
            s.shape[a] = n
        s.n_channels = self.n_channels
        s.n_levels = self.n_levels
        for l, P in enumerate(self.max_disp[:MAX_LEVELS]):
            s.max_disp[l] = P
        for l, w in enumerate(self.level_weight[:MAX_LEVELS]):
            s.level_weight[l] = w
        s.n_pairs = len(self.pairs)
        for q, (i, j) in enumerate(self.pairs):
            s.pairs[2 * q] = i
            s.pairs[2 * q + 1] = j
        s.path = self.path
        s.flags = self.flags
        s.descriptor = self.descriptor
        s.s3_max_disp = self.s3_max_disp
        s.alpha = self.alpha
        return s


def make_spec(shape, n_channels=1, n_levels=1, P=16, **kw) -> Spec:
    """A spec with the same P on every level (the library clips it per level)."""
    return Spec(shape=tuple(shape), n_channels=n_channels, n_levels=n_levels,
                max_disp=(int(P),) * max(1, n_levels), **kw)


# ---------------------------------------------------------------------------
_lib = None
_vp = ctypes.c_void_p


def lib():
    """Load libdmcr.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdmcr.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2103_09686_amd.build_lib)")
        L = ctypes.CDLL(LIB_PATH)
        sp = ctypes.POINTER(c_spec)
        L.dmcr_descriptor_size.argtypes = [sp]
        L.dmcr_descriptor_size.restype = ctypes.c_int64
        L.dmcr_level_count.argtypes = [sp]
        L.dmcr_level_count.restype = ctypes.c_int32
        L.dmcr_descriptor_offsets.argtypes = [sp, ctypes.POINTER(ctypes.c_int64)]
        L.dmcr_workspace_size.argtypes = [sp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.dmcr_pyramid.argtypes = [sp, ctypes.c_int32, _vp, _vp, _vp]
        L.dmcr_descriptor_forward.argtypes = [sp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.dmcr_descriptor_adjoint.argtypes = [sp, ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.dmcr_error_cotangent.argtypes = [sp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.dmcr_loss_grad.argtypes = [sp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.dmcr_penalised_loss_grad.argtypes = [sp, ctypes.c_int32, _vp, _vp, ctypes.POINTER(c_bounds), _vp, _vp, _vp,
                                               _vp, ctypes.c_size_t, _vp]
        L.dmcr_reconstruct_workspace_size.argtypes = [sp, ctypes.c_int32, ctypes.POINTER(c_opt),
                                                      ctypes.POINTER(ctypes.c_size_t)]
        L.dmcr_reconstruct.argtypes = [sp, ctypes.c_int32, _vp, ctypes.POINTER(c_bounds),
                                       ctypes.POINTER(c_opt), _vp, ctypes.POINTER(c_result), _vp,
                                       ctypes.c_size_t, _vp]
        L.dmcr_reconstruct_c2f_workspace_size.argtypes = [sp, ctypes.c_int32, ctypes.POINTER(c_opt),
                                                          ctypes.POINTER(ctypes.c_size_t)]
        L.dmcr_reconstruct_coarse_to_fine.argtypes = [sp, ctypes.c_int32, _vp, ctypes.POINTER(c_bounds),
                                                      ctypes.POINTER(c_opt), _vp, ctypes.POINTER(c_result), _vp,
                                                      ctypes.c_size_t, _vp]
        L.dmcr_solver_start.argtypes = [sp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, _vp,
                                        ctypes.POINTER(c_bounds), ctypes.POINTER(c_opt), _vp,
                                        ctypes.POINTER(c_slot), _vp, ctypes.c_size_t, _vp]
        L.dmcr_solver_iterate.argtypes = [sp, ctypes.c_int32, _vp, ctypes.POINTER(c_bounds), ctypes.POINTER(c_opt),
                                          _vp, ctypes.POINTER(c_slot), ctypes.POINTER(c_ring), ctypes.c_int32, _vp,
                                          ctypes.c_size_t, _vp]
        L.dmcr_status_string.argtypes = [ctypes.c_int]
        L.dmcr_status_string.restype = ctypes.c_char_p
        for fn in ("dmcr_descriptor_offsets", "dmcr_workspace_size", "dmcr_pyramid",
                   "dmcr_descriptor_forward", "dmcr_descriptor_adjoint", "dmcr_error_cotangent",
                   "dmcr_loss_grad", "dmcr_penalised_loss_grad", "dmcr_reconstruct_workspace_size", "dmcr_reconstruct",
                   "dmcr_reconstruct_c2f_workspace_size", "dmcr_reconstruct_coarse_to_fine",
                   "dmcr_solver_start", "dmcr_solver_iterate"):
            getattr(L, fn).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(fn, code):
    if code < 0:
        raise DmcrError(fn, code)
    return code


def _stream(stream=None, *own):
    """The HIP stream of a call.  When it is not the current stream, it first waits
    for the current one (which produced the inputs and on which the binding's own
    buffers `own` were allocated), and those buffers are marked as used by it, so
    that the caching allocator does not hand their memory out before it is done."""
    cur = torch.cuda.current_stream()
    if stream is None or stream == cur:
        return ctypes.c_void_p(cur.cuda_stream)
    stream.wait_stream(cur)
    for t in own:
        if t is not None:
            t.record_stream(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor, dtype, what):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % what)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (what, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return ctypes.c_void_p(t.data_ptr())


def dmcr_descriptor_size(spec: Spec) -> int:
    s = spec.c()
    return _check("dmcr_descriptor_size", lib().dmcr_descriptor_size(ctypes.byref(s)))


def dmcr_level_count(spec: Spec) -> int:
    s = spec.c()
    return _check("dmcr_level_count", lib().dmcr_level_count(ctypes.byref(s)))


def dmcr_descriptor_offsets(spec: Spec):
    s = spec.c()
    n = dmcr_level_count(spec) * (len(spec.pairs) + (spec.n_channels if spec.s3_max_disp > 0 else 0)) + 1
    out = (ctypes.c_int64 * n)()
    _check("dmcr_descriptor_offsets", lib().dmcr_descriptor_offsets(ctypes.byref(s), out))
    return list(out)


def dmcr_workspace_size(spec: Spec, batch: int) -> int:
    s = spec.c()
    b = ctypes.c_size_t()
    _check("dmcr_workspace_size", lib().dmcr_workspace_size(ctypes.byref(s), batch, ctypes.byref(b)))
    return b.value


def workspace(nbytes: int, device=None) -> torch.Tensor:
    """A 256-byte-aligned uint8 device buffer of at least nbytes."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    buf = torch.empty(max(1, nbytes) + 256, dtype=torch.uint8, device=dev)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + max(1, nbytes)]


def _batch(spec: Spec, phi: torch.Tensor):
    if phi.dim() != spec.ndim + 2 or tuple(phi.shape[2:]) != spec.shape or phi.shape[1] != spec.n_channels:
        raise ValueError("phi must be [B][%d]%s, got %s" % (spec.n_channels, list(spec.shape), tuple(phi.shape)))
    return int(phi.shape[0])


def _ws(spec, B, ws, phi, own=None):
    """The caller's workspace, or a new one (appended to `own`, the binding's buffers)."""
    need = dmcr_workspace_size(spec, B)
    if ws is None:
        ws = workspace(need, phi.device)
        if own is not None:
            own.append(ws)
    if ws.numel() < need:
        raise ValueError("workspace of %d bytes < %d" % (ws.numel(), need))
    return ws, need


def dmcr_pyramid(spec: Spec, phi: torch.Tensor, stream=None):
    """Levels 1..L-1 of the mean-pool pyramid, as a list of tensors."""
    B = _batch(spec, phi)
    sizes = [B * spec.n_channels * (int(torch.tensor([s >> l for s in spec.shape]).prod()))
             for l in range(1, dmcr_level_count(spec))]
    out = torch.empty(max(1, sum(sizes)), dtype=torch.float32, device=phi.device)
    s = spec.c()
    _check("dmcr_pyramid", lib().dmcr_pyramid(ctypes.byref(s), B, _ptr(phi, torch.float32, "phi"),
                                              ctypes.c_void_p(out.data_ptr()), _stream(stream, out)))
    res, o = [], 0
    for l, n in enumerate(sizes, start=1):
        res.append(out[o:o + n].view((B, spec.n_channels) + tuple(x >> l for x in spec.shape)))
        o += n
    return res


def dmcr_descriptor_forward(spec: Spec, phi: torch.Tensor, S: Optional[torch.Tensor] = None,
                            ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    B = _batch(spec, phi)
    K = dmcr_descriptor_size(spec)
    own = []
    if S is None:
        S = torch.empty((B, K), dtype=torch.float32, device=phi.device)
        own.append(S)
    ws, need = _ws(spec, B, ws, phi, own)
    s = spec.c()
    _check("dmcr_descriptor_forward", lib().dmcr_descriptor_forward(
        ctypes.byref(s), B, _ptr(phi, torch.float32, "phi"), _ptr(S, torch.float32, "S"),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream, *own)))
    return S


def dmcr_descriptor_adjoint(spec: Spec, phi: torch.Tensor, dS: torch.Tensor,
                            grad: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                            stream=None) -> torch.Tensor:
    B = _batch(spec, phi)
    own = []
    if grad is None:
        grad = torch.empty_like(phi)
        own.append(grad)
    ws, need = _ws(spec, B, ws, phi, own)
    s = spec.c()
    _check("dmcr_descriptor_adjoint", lib().dmcr_descriptor_adjoint(
        ctypes.byref(s), B, _ptr(phi, torch.float32, "phi"), _ptr(dS, torch.float32, "dS"),
        _ptr(grad, torch.float32, "grad"), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream, *own)))
    return grad


def dmcr_error_cotangent(spec: Spec, S: torch.Tensor, S_target: torch.Tensor, E=None, G=None,
                         ws=None, stream=None):
    B = int(S.shape[0])
    own = []
    if E is None:
        E = torch.empty(B, dtype=torch.float64, device=S.device)
        own.append(E)
    if G is None:
        G = torch.empty_like(S)
        own.append(G)
    ws, need = _ws(spec, B, ws, S, own)
    s = spec.c()
    _check("dmcr_error_cotangent", lib().dmcr_error_cotangent(
        ctypes.byref(s), B, _ptr(S, torch.float32, "S"), _ptr(S_target, torch.float64, "S_target"),
        _ptr(E, torch.float64, "E"), _ptr(G, torch.float32, "G"), ctypes.c_void_p(ws.data_ptr()),
        ws.numel(), _stream(stream, *own)))
    return E, G


def dmcr_loss_grad(spec: Spec, phi: torch.Tensor, S_target: torch.Tensor, E=None, grad=None, ws=None,
                   stream=None):
    B = _batch(spec, phi)
    own = []
    if E is None:
        E = torch.empty(B, dtype=torch.float64, device=phi.device)
        own.append(E)
    if grad is None:
        grad = torch.empty_like(phi)
        own.append(grad)
    ws, need = _ws(spec, B, ws, phi, own)
    s = spec.c()
    _check("dmcr_loss_grad", lib().dmcr_loss_grad(
        ctypes.byref(s), B, _ptr(phi, torch.float32, "phi"), _ptr(S_target, torch.float64, "S_target"),
        _ptr(E, torch.float64, "E"), _ptr(grad, torch.float32, "grad"), ctypes.c_void_p(ws.data_ptr()),
        ws.numel(), _stream(stream, *own)))
    return E, grad


def dmcr_penalised_loss_grad(spec: Spec, phi: torch.Tensor, S_target: torch.Tensor, bounds: "Bounds",
                             L=None, E=None, grad=None, ws=None, stream=None):
    """(L, E, grad) of the relaxed problem's loss; see include/dmcr.h."""
    B = _batch(spec, phi)
    own = []
    if L is None:
        L = torch.empty(B, dtype=torch.float64, device=phi.device)
        own.append(L)
    if E is None:
        E = torch.empty(B, dtype=torch.float64, device=phi.device)
        own.append(E)
    if grad is None:
        grad = torch.empty_like(phi)
        own.append(grad)
    ws, need = _ws(spec, B, ws, phi, own)
    s, bo = spec.c(), bounds.c()
    _check("dmcr_penalised_loss_grad", lib().dmcr_penalised_loss_grad(
        ctypes.byref(s), B, _ptr(phi, torch.float32, "phi"), _ptr(S_target, torch.float64, "S_target"),
        ctypes.byref(bo), _ptr(L, torch.float64, "L"), _ptr(E, torch.float64, "E"), _ptr(grad, torch.float32, "grad"),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream, *own)))
    return L, E, grad


@dataclass
class Bounds:
    lo: float = 0.0
    hi: float = 1.0
    mode: int = BOUNDS_PROJECT
    kappa: float = 1.0

    def c(self):
        return c_bounds(self.lo, self.hi, self.mode, self.kappa)


@dataclass
class Opt:
    """Optimizer settings (dmcr_opt): L-BFGS by default; method=OPT_ADAM selects Adam
    with the paper's TensorFlow defaults lr 1e-3, betas 0.9 / 0.999, eps 1e-7."""
    m: int = 10
    max_iter: int = 100
    max_ls: int = 20
    tol_derr: float = 1e-4
    c1: float = 1e-4
    method: int = 0
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-7

    def c(self):
        return c_opt(self.m, self.max_iter, self.max_ls, self.tol_derr, self.c1, self.method,
                     self.lr, self.beta1, self.beta2, self.eps)


def dmcr_reconstruct_workspace_size(spec: Spec, batch: int, opt: Opt) -> int:
    s, o = spec.c(), opt.c()
    b = ctypes.c_size_t()
    _check("dmcr_reconstruct_workspace_size",
           lib().dmcr_reconstruct_workspace_size(ctypes.byref(s), batch, ctypes.byref(o), ctypes.byref(b)))
    return b.value


def dmcr_reconstruct(spec: Spec, S_target: torch.Tensor, phi: torch.Tensor, bounds: Bounds = None,
                     opt: Opt = None, ws=None, stream=None):
    """Runs L-BFGS in place on phi ([B][C][n...]); returns a list of result dicts."""
    bounds = bounds or Bounds()
    opt = opt or Opt()
    B = _batch(spec, phi)
    need = dmcr_reconstruct_workspace_size(spec, B, opt)
    own = []
    if ws is None:
        ws = workspace(need, phi.device)
        own.append(ws)
    s, bo, o = spec.c(), bounds.c(), opt.c()
    res = (c_result * B)()
    code = lib().dmcr_reconstruct(ctypes.byref(s), B, _ptr(S_target, torch.float64, "S_target"),
                                  ctypes.byref(bo), ctypes.byref(o), _ptr(phi, torch.float32, "phi"), res,
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream, *own))
    _check("dmcr_reconstruct", code)
    return code, [dict(final_E=r.final_E, final_derr=r.final_derr, iters=r.iters, evals=r.evals, why=r.why)
                  for r in res]


def dmcr_reconstruct_c2f_workspace_size(spec: Spec, batch: int, opt: Opt) -> int:
    s, o = spec.c(), opt.c()
    b = ctypes.c_size_t()
    _check("dmcr_reconstruct_c2f_workspace_size",
           lib().dmcr_reconstruct_c2f_workspace_size(ctypes.byref(s), batch, ctypes.byref(o), ctypes.byref(b)))
    return b.value


def dmcr_reconstruct_coarse_to_fine(spec: Spec, S_target: torch.Tensor, phi: torch.Tensor, bounds: Bounds = None,
                                    opt: Opt = None, ws=None, stream=None):
    """Sequential coarse-to-fine reconstruction in place on phi (level by level,
    coarsest first, each started from the upsampled result of the coarser level);
    returns (code, list of result dicts) with the multigrid error of the result."""
    bounds = bounds or Bounds()
    opt = opt or Opt()
    B = _batch(spec, phi)
    need = dmcr_reconstruct_c2f_workspace_size(spec, B, opt)
    own = []
    if ws is None:
        ws = workspace(need, phi.device)
        own.append(ws)
    s, bo, o = spec.c(), bounds.c(), opt.c()
    res = (c_result * B)()
    code = lib().dmcr_reconstruct_coarse_to_fine(ctypes.byref(s), B, _ptr(S_target, torch.float64, "S_target"),
                                                 ctypes.byref(bo), ctypes.byref(o), _ptr(phi, torch.float32, "phi"),
                                                 res, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                                 _stream(stream, *own))
    _check("dmcr_reconstruct_coarse_to_fine", code)
    return code, [dict(final_E=r.final_E, final_derr=r.final_derr, iters=r.iters, evals=r.evals, why=r.why)
                  for r in res]


class Solver:
    """A batch of `batch` L-BFGS slots of one spec for continuous batching
    (dmcr_solver_start / dmcr_solver_iterate).  Holds the field and target
    buffers, the workspace, the host slot array and the history ring."""

    def __init__(self, spec: Spec, batch: int, bounds: Bounds = None, opt: Opt = None, device=None, stream=None):
        """With `stream`, the buffers are allocated and cleared in that stream's order
        (the stream the solver's calls will then run on)."""
        self.spec, self.B = spec, batch
        self.bounds, self.opt = bounds or Bounds(), opt or Opt()
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.K = dmcr_descriptor_size(spec)
        self.ws_bytes = dmcr_reconstruct_workspace_size(spec, batch, self.opt)
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            self.phi = torch.zeros((batch, spec.n_channels) + tuple(spec.shape), dtype=torch.float32, device=dev)
            self.St = torch.zeros((batch, self.K), dtype=torch.float64, device=dev)
            self.ws = workspace(self.ws_bytes, dev)
        self.slots = (c_slot * batch)()
        self.ring = c_ring(self.opt.m - 1, 0)
        self._c = (spec.c(), self.bounds.c(), self.opt.c())

    @property
    def footprint(self) -> int:
        return self.phi.numel() * 4 + self.St.numel() * 8 + self.ws.numel()

    def start(self, which, stream=None):
        idx = (ctypes.c_int32 * len(which))(*which)
        s, b, o = self._c
        _check("dmcr_solver_start", lib().dmcr_solver_start(
            ctypes.byref(s), self.B, idx, len(which), ctypes.c_void_p(self.St.data_ptr()), ctypes.byref(b),
            ctypes.byref(o), ctypes.c_void_p(self.phi.data_ptr()), self.slots, ctypes.c_void_p(self.ws.data_ptr()),
            self.ws.numel(), _stream(stream)))

    def iterate(self, iterations: int, stream=None, trace: list = None):
        """Up to `iterations` iterations of every running slot.  With `trace` (a list),
        the iterations run one call at a time and each slot that took one appends a
        record: dict(slot, iters, evals, E, f, status), its state after that iteration
        (per-iteration metrics; a call synchronises the device anyway)."""
        s, b, o = self._c
        steps = [iterations] if trace is None else [1] * iterations
        for n in steps:
            before = [self.slots[i].iters for i in range(self.B)]
            _check("dmcr_solver_iterate", lib().dmcr_solver_iterate(
                ctypes.byref(s), self.B, ctypes.c_void_p(self.St.data_ptr()), ctypes.byref(b), ctypes.byref(o),
                ctypes.c_void_p(self.phi.data_ptr()), self.slots, ctypes.byref(self.ring), n,
                ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), _stream(stream)))
            if trace is not None:
                for i in range(self.B):
                    sl = self.slots[i]
                    if sl.iters != before[i]:
                        trace.append(dict(slot=i, iters=sl.iters, evals=sl.evals, E=sl.E, f=sl.f, status=sl.status))

    def state_dict(self) -> dict:
        """A host copy of the whole solver state, for checkpoint and resume: fields,
        targets, the workspace (history ring, step data, counters; it holds offsets,
        no addresses, so it may be restored at any address), the slot array and the
        ring cursor.  A solver of the same spec, batch, bounds and settings that loads
        it continues bitwise as this one would.  Synchronises the device."""
        torch.cuda.synchronize(self.phi.device)
        return dict(spec=self.spec, batch=self.B, bounds=self.bounds, opt=self.opt, ws_bytes=self.ws_bytes,
                    phi=self.phi.cpu(), St=self.St.cpu(), ws=self.ws.cpu(),
                    slots=ctypes.string_at(ctypes.addressof(self.slots), ctypes.sizeof(self.slots)),
                    ring=ctypes.string_at(ctypes.addressof(self.ring), ctypes.sizeof(self.ring)))

    def load_state_dict(self, state: dict):
        """Restore a state taken by state_dict() (of this solver or another one of the
        same spec, batch, bounds and settings)."""
        mine = (self.spec, self.B, self.bounds, self.opt, self.ws_bytes)
        theirs = (state["spec"], state["batch"], state["bounds"], state["opt"], state["ws_bytes"])
        if mine != theirs:
            raise ValueError("checkpoint of a different solver (spec, batch, bounds, settings or workspace)")
        if len(state["slots"]) != ctypes.sizeof(self.slots) or len(state["ring"]) != ctypes.sizeof(self.ring):
            raise ValueError("checkpoint slot array or ring cursor of the wrong size")
        self.phi.copy_(state["phi"])
        self.St.copy_(state["St"])
        self.ws.copy_(state["ws"])
        torch.cuda.synchronize(self.phi.device)
        ctypes.memmove(ctypes.addressof(self.slots), state["slots"], len(state["slots"]))
        ctypes.memmove(ctypes.addressof(self.ring), state["ring"], len(state["ring"]))


class S2Descriptor(torch.autograd.Function):
    """phi [B][C][n...] -> S [B][K]; backward runs dmcr_descriptor_adjoint (spectra recomputed)."""

    @staticmethod
    def forward(ctx, phi, spec):
        phi = phi.contiguous()
        ctx.spec = spec
        ctx.save_for_backward(phi)
        return dmcr_descriptor_forward(spec, phi)

    @staticmethod
    def backward(ctx, dS):
        (phi,) = ctx.saved_tensors
        g = dmcr_descriptor_adjoint(ctx.spec, phi, dS.contiguous().to(torch.float32))
        return g, None


def s2_descriptor(phi, spec):
    return S2Descriptor.apply(phi, spec)
