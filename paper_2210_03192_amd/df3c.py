"""Python binding of libdf3c (ctypes).  Argument marshalling only: every step
of the integral path runs in the library's HIP kernels; PyTorch provides the
device memory and the stream.  There is no CPU fallback: without the built
library (or without a GPU) these functions raise.
"""
import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# DF3C_LIBRARY selects another build of the library (e.g. a tuning variant)
LIB_PATH = os.environ.get("DF3C_LIBRARY") or os.path.join(_HERE, "libdf3c.so")
_lib = None

DF3C_OK = 0
SCHED_PER_CLASS = 0
SCHED_PERSISTENT = 1
GRAPH = 2
ASYNC = 4
NCLASS = 175


class ClassTune(ctypes.Structure):
    """Per-class schedule parameters of the persistent batched J."""
    _fields_ = [("chunk", ctypes.c_int32), ("grid_per_cu", ctypes.c_int32),
                ("enabled", ctypes.c_int32), ("order", ctypes.c_int32)]


def class_index(lp: int, la: int, lb: int) -> int:
    return (lp * 5 + la) * 5 + lb


def default_tune():
    t = (ClassTune * NCLASS)()
    for c in range(NCLASS):
        t[c] = ClassTune(1, 4, 1, -(c // 25))
    return t


class DF3CError(RuntimeError):
    pass


class _Shells(ctypes.Structure):
    _fields_ = [
        ("nshell", ctypes.c_int32),
        ("l_host", ctypes.c_void_p),
        ("l", ctypes.c_void_p),
        ("nprim", ctypes.c_void_p),
        ("prim_off", ctypes.c_void_p),
        ("atom", ctypes.c_void_p),
        ("exps", ctypes.c_void_p),
        ("coefs", ctypes.c_void_p),
        ("pure", ctypes.c_int32),
        ("nprim_host", ctypes.c_void_p),
    ]


def lib():
    """The loaded libdf3c (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DF3CError(f"{LIB_PATH} is missing: build it with paper_2210_03192_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, U32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
        L.df3c_init.argtypes = []
        L.df3c_workspace_status.argtypes = [P, P]
        L.df3c_status_string.restype = ctypes.c_char_p
        L.df3c_status_string.argtypes = [ctypes.c_int]
        L.df3c_eval_batch_workspace.restype = SZ
        L.df3c_eval_batch_workspace.argtypes = [I64]
        I32 = ctypes.c_int32
        L.df3c_eval_batch.argtypes = [P, I32, P, P, I64, P, P, P, P, SZ, U32, P]
        L.df3c_coulomb_J_workspace.restype = SZ
        L.df3c_coulomb_J_workspace.argtypes = [P, P]
        L.df3c_coulomb_J.argtypes = [P, I32, P, P, P, P, P, SZ, U32, P]
        L.df3c_screen_pairs.argtypes = [P, I32, P, ctypes.c_double, P, P]
        L.df3c_screen_pairs_schwarz_workspace.restype = SZ
        L.df3c_screen_pairs_schwarz_workspace.argtypes = []
        L.df3c_screen_pairs_schwarz.argtypes = [P, I32, P, P, P, ctypes.c_double, P, P, SZ, U32, P]
        L.df3c_coulomb_J_masked_workspace.restype = SZ
        L.df3c_coulomb_J_masked_workspace.argtypes = [P, P]
        L.df3c_coulomb_J_masked.argtypes = [P, I32, P, P, P, P, P, P, SZ, U32, P]
        L.df3c_coulomb_J_grad_workspace.restype = SZ
        L.df3c_coulomb_J_grad_workspace.argtypes = [P, P, I32]
        L.df3c_coulomb_J_grad.argtypes = [P, I32, P, P, P, P, P, P, SZ, U32, P]
        L.df3c_coulomb_J_grad_masked_workspace.restype = SZ
        L.df3c_coulomb_J_grad_masked_workspace.argtypes = [P, P, I32]
        L.df3c_coulomb_J_grad_masked.argtypes = [P, I32, P, P, P, P, P, P, P, SZ, U32, P]
        L.df3c_coulomb_J_grad_batched_workspace.restype = SZ
        L.df3c_coulomb_J_grad_batched_workspace.argtypes = [P, P, I32, P, P, P]
        L.df3c_coulomb_J_grad_batched.argtypes = [P, I32, P, P, I32, P, P, P, P, P, P, P, SZ,
                                                  U32, P]
        L.df3c_coulomb_J_batched_workspace.restype = SZ
        L.df3c_coulomb_J_batched_workspace.argtypes = [P, P, I32, P]
        L.df3c_coulomb_J_batched.argtypes = [P, I32, P, P, I32, P, P, P, P, P, P, SZ, U32, P]
        L.df3c_coulomb_metric_workspace.restype = SZ
        L.df3c_coulomb_metric_workspace.argtypes = [P]
        L.df3c_coulomb_metric.argtypes = [P, I32, P, P, P, SZ, U32, P]
        L.df3c_coulomb_gamma_workspace.restype = SZ
        L.df3c_coulomb_gamma_workspace.argtypes = [P, P]
        L.df3c_coulomb_gamma.argtypes = [P, I32, P, P, P, P, P, SZ, U32, P]
        L.df3c_fit_solve_workspace.restype = SZ
        L.df3c_fit_solve_workspace.argtypes = [I64]
        L.df3c_fit_solve.argtypes = [P, I64, P, P, P, SZ, U32, P]
        L.df3c_timing_enable.argtypes = [I32]
        L.df3c_timing_read.restype = I64
        L.df3c_timing_read.argtypes = [P, P, P, I64]
        _lib = L
    return _lib


def _check(rc, what):
    if rc != DF3C_OK:
        raise DF3CError(f"{what}: {lib().df3c_status_string(rc).decode()} (status {rc})")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


@dataclass
class DeviceBasis:
    """A basis resident on the GPU (arrays of paper_2210_03192_amd.inputs.Basis)."""
    l_host: np.ndarray
    l: torch.Tensor
    nprim: torch.Tensor
    prim_off: torch.Tensor
    atom: torch.Tensor
    exps: torch.Tensor
    coefs: torch.Tensor
    pure: int
    nprim_host: Optional[np.ndarray] = None   # host copy of nprim (orders pairs)

    @classmethod
    def from_basis(cls, b, device="cuda"):
        l_host = np.ascontiguousarray(b.l, np.int32)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
        return cls(l_host, t(b.l, torch.int32), t(b.nprim, torch.int32),
                   t(b.prim_off, torch.int64), t(b.atom, torch.int32),
                   t(b.exps, torch.float64), t(b.coefs, torch.float64), int(b.pure),
                   np.ascontiguousarray(b.nprim, np.int32))

    @property
    def nshell(self):
        return int(self.l_host.shape[0])

    def struct(self):
        return _Shells(self.nshell, self.l_host.ctypes.data, self.l.data_ptr(),
                       self.nprim.data_ptr(), self.prim_off.data_ptr(), self.atom.data_ptr(),
                       self.exps.data_ptr(), self.coefs.data_ptr(), self.pure,
                       None if self.nprim_host is None else self.nprim_host.ctypes.data)

    def offsets(self):
        n = np.array([2 * l + 1 if self.pure else (l + 1) * (l + 2) // 2 for l in self.l_host],
                     np.int64)
        return np.concatenate([[0], np.cumsum(n)]).astype(np.int64)


def init():
    _check(lib().df3c_init(), "df3c_init")


def workspace_status(ws: torch.Tensor, stream=None) -> int:
    """Status of the last call that used ws (synchronises the stream); for
    calls made with ASYNC."""
    return int(lib().df3c_workspace_status(_ptr(ws), _stream(stream)))


def check_workspace(ws: torch.Tensor, what: str, stream=None) -> None:
    """Raise DF3CError if the last call that used ws failed on the device."""
    _check(workspace_status(ws, stream), what)


def eval_batch_workspace(ntrip: int) -> int:
    return int(lib().df3c_eval_batch_workspace(int(ntrip)))


def eval_batch(xyz: torch.Tensor, aux: DeviceBasis, orb: DeviceBasis, trip: torch.Tensor,
               out_off: torch.Tensor, out: torch.Tensor, ws: Optional[torch.Tensor] = None,
               flags: int = 0, stream=None) -> torch.Tensor:
    """(P|ab) blocks of trip[t] = (P, a, b) written to out[out_off[t]:]."""
    ntrip = int(trip.shape[0])
    need = eval_batch_workspace(ntrip)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=xyz.device)
    sa, so = aux.struct(), orb.struct()
    _check(lib().df3c_eval_batch(_ptr(xyz), int(xyz.shape[0]), ctypes.byref(sa), ctypes.byref(so),
                                 ntrip, _ptr(trip),
                                 _ptr(out_off), _ptr(out), _ptr(ws), ws.numel(), flags,
                                 _stream(stream)), "df3c_eval_batch")
    return out


def coulomb_J_workspace(aux: DeviceBasis, orb: DeviceBasis) -> int:
    sa, so = aux.struct(), orb.struct()
    return int(lib().df3c_coulomb_J_workspace(ctypes.byref(sa), ctypes.byref(so)))


def coulomb_J(xyz: torch.Tensor, aux: DeviceBasis, orb: DeviceBasis, d: torch.Tensor,
              J: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
              flags: int = 0, stream=None) -> torch.Tensor:
    """J_ab = sum_P (ab|P) d_P (both triangles)."""
    nao = int(orb.offsets()[-1])
    if J is None:
        J = torch.empty((nao, nao), dtype=torch.float64, device=xyz.device)
    need = coulomb_J_workspace(aux, orb)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=xyz.device)
    sa, so = aux.struct(), orb.struct()
    _check(lib().df3c_coulomb_J(_ptr(xyz), int(xyz.shape[0]), ctypes.byref(sa), ctypes.byref(so),
                                _ptr(d), _ptr(J), _ptr(ws), ws.numel(), flags, _stream(stream)),
           "df3c_coulomb_J")
    return J


def screen_pairs(xyz: torch.Tensor, orb: DeviceBasis, tau: float, mask: Optional[torch.Tensor] = None,
                 stream=None) -> torch.Tensor:
    """Shell-pair mask (nshell x nshell, uint8, symmetric): 1 where the largest
    primitive overlap bound of the pair is >= tau."""
    n = orb.nshell
    if mask is None:
        mask = torch.empty((n, n), dtype=torch.uint8, device=xyz.device)
    so = orb.struct()
    _check(lib().df3c_screen_pairs(_ptr(xyz), int(xyz.shape[0]), ctypes.byref(so), float(tau),
                                   _ptr(mask), _stream(stream)), "df3c_screen_pairs")
    return mask


def screen_pairs_schwarz(xyz: torch.Tensor, aux: DeviceBasis, orb: DeviceBasis, d: torch.Tensor,
                         tau: float, mask: Optional[torch.Tensor] = None, flags: int = 0,
                         stream=None) -> torch.Tensor:
    """Shell-pair mask with the Schwarz-type error guarantee: 1 where
    Q_ab S_d >= tau (every element of a dropped pair's J block is below tau)."""
    n = orb.nshell
    if mask is None:
        mask = torch.empty((n, n), dtype=torch.uint8, device=xyz.device)
    ws = torch.empty(int(lib().df3c_screen_pairs_schwarz_workspace()), dtype=torch.uint8,
                     device=xyz.device)
    sa, so = aux.struct(), orb.struct()
    _check(lib().df3c_screen_pairs_schwarz(_ptr(xyz), int(xyz.shape[0]), ctypes.byref(sa),
                                           ctypes.byref(so), _ptr(d), float(tau), _ptr(mask),
                                           _ptr(ws), ws.numel(), flags, _stream(stream)),
           "df3c_screen_pairs_schwarz")
    return mask


def coulomb_J_masked_workspace(aux: DeviceBasis, orb: DeviceBasis) -> int:
    sa, so = aux.struct(), orb.struct()
    return int(lib().df3c_coulomb_J_masked_workspace(ctypes.byref(sa), ctypes.byref(so)))


def coulomb_J_masked(xyz: torch.Tensor, aux: DeviceBasis, orb: DeviceBasis, d: torch.Tensor,
                     mask: torch.Tensor, J: Optional[torch.Tensor] = None,
                     ws: Optional[torch.Tensor] = None, flags: int = 0, stream=None) -> torch.Tensor:
    """J over the shell pairs the mask keeps (the other blocks zero)."""
    nao = int(orb.offsets()[-1])
    if J is None:
        J = torch.empty((nao, nao), dtype=torch.float64, device=xyz.device)
    need = coulomb_J_masked_workspace(aux, orb)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=xyz.device)
    sa, so = aux.struct(), orb.struct()
    _check(lib().df3c_coulomb_J_masked(_ptr(xyz), int(xyz.shape[0]), ctypes.byref(sa),
                                       ctypes.byref(so), _ptr(d), _ptr(mask), _ptr(J), _ptr(ws),
                                       ws.numel(), flags, _stream(stream)),
           "df3c_coulomb_J_masked")
    return J


def coulomb_J_grad_masked_workspace(aux: DeviceBasis, orb: DeviceBasis, natom: int) -> int:
    sa, so = aux.struct(), orb.struct()
    return int(lib().df3c_coulomb_J_grad_masked_workspace(ctypes.byref(sa), ctypes.byref(so),
                                                          int(natom)))


def coulomb_J_grad_masked(xyz: torch.Tensor, aux: DeviceBasis, orb: DeviceBasis, d: torch.Tensor,
                          G: torch.Tensor, mask: torch.Tensor, grad: Optional[torch.Tensor] = None,
                          ws: Optional[torch.Tensor] = None, flags: int = 0,
                          stream=None) -> torch.Tensor:
    """dL/dR [natom][3] of L = sum_ab G_ab J_ab over the shell pairs the mask keeps."""
    natom = int(xyz.shape[0])
    if grad is None:
        grad = torch.empty((natom, 3), dtype=torch.float64, device=xyz.device)
    need = coulomb_J_grad_masked_workspace(aux, orb, natom)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=xyz.device)
    G = G.contiguous()
    sa, so = aux.struct(), orb.struct()
    _check(lib().df3c_coulomb_J_grad_masked(_ptr(xyz), natom, ctypes.byref(sa), ctypes.byref(so),
                                            _ptr(d), _ptr(G), _ptr(mask), _ptr(grad), _ptr(ws),
                                            ws.numel(), flags, _stream(stream)),
           "df3c_coulomb_J_grad_masked")
    return grad


def coulomb_J_grad_workspace(aux: DeviceBasis, orb: DeviceBasis, natom: int) -> int:
    sa, so = aux.struct(), orb.struct()
    return int(lib().df3c_coulomb_J_grad_workspace(ctypes.byref(sa), ctypes.byref(so), int(natom)))


def coulomb_J_grad(xyz: torch.Tensor, aux: DeviceBasis, orb: DeviceBasis, d: torch.Tensor,
                   G: torch.Tensor, grad: Optional[torch.Tensor] = None,
                   ws: Optional[torch.Tensor] = None, flags: int = 0, stream=None) -> torch.Tensor:
    """dL/dxyz for L = sum_ab G_ab J_ab (d and G fixed)."""
    natom = int(xyz.shape[0])
    if grad is None:
        grad = torch.empty((natom, 3), dtype=torch.float64, device=xyz.device)
    need = coulomb_J_grad_workspace(aux, orb, natom)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=xyz.device)
    G = G.contiguous()
    sa, so = aux.struct(), orb.struct()
    _check(lib().df3c_coulomb_J_grad(_ptr(xyz), natom, ctypes.byref(sa), ctypes.byref(so), _ptr(d),
                                     _ptr(G), _ptr(grad), _ptr(ws), ws.numel(), flags,
                                     _stream(stream)), "df3c_coulomb_J_grad")
    return grad


def coulomb_metric(xyz: torch.Tensor, aux: DeviceBasis, V: Optional[torch.Tensor] = None,
                   ws: Optional[torch.Tensor] = None, flags: int = 0, stream=None) -> torch.Tensor:
    """V[P][Q] = (P|Q), the two-centre metric of the aux basis."""
    naux = int(aux.offsets()[-1])
    if V is None:
        V = torch.empty((naux, naux), dtype=torch.float64, device=xyz.device)
    sa = aux.struct()
    need = int(lib().df3c_coulomb_metric_workspace(ctypes.byref(sa)))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=xyz.device)
    _check(lib().df3c_coulomb_metric(_ptr(xyz), int(xyz.shape[0]), ctypes.byref(sa), _ptr(V),
                                     _ptr(ws), ws.numel(), flags, _stream(stream)),
           "df3c_coulomb_metric")
    return V


def coulomb_gamma_workspace(aux: DeviceBasis, orb: DeviceBasis) -> int:
    return int(lib().df3c_coulomb_gamma_workspace(ctypes.byref(aux.struct()),
                                                  ctypes.byref(orb.struct())))


def coulomb_gamma(xyz: torch.Tensor, aux: DeviceBasis, orb: DeviceBasis, D: torch.Tensor,
                  gamma: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                  flags: int = 0, stream=None) -> torch.Tensor:
    """gamma_P = sum_{a,b} (P|ab) D_ab (D: nao x nao, any symmetry)."""
    naux = int(aux.offsets()[-1])
    if gamma is None:
        gamma = torch.empty(naux, dtype=torch.float64, device=xyz.device)
    need = coulomb_gamma_workspace(aux, orb)
    if need == 0:
        raise DF3CError("df3c_coulomb_gamma_workspace failed")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=xyz.device)
    sa, so = aux.struct(), orb.struct()
    _check(lib().df3c_coulomb_gamma(_ptr(xyz), int(xyz.shape[0]), ctypes.byref(sa),
                                    ctypes.byref(so), _ptr(D), _ptr(gamma), _ptr(ws), ws.numel(),
                                    flags, _stream(stream)), "df3c_coulomb_gamma")
    return gamma


def fit_solve(V: torch.Tensor, rhs: torch.Tensor, x: Optional[torch.Tensor] = None,
              ws: Optional[torch.Tensor] = None, flags: int = 0, stream=None) -> torch.Tensor:
    """x = V^{-1} rhs by the library's Cholesky (V is overwritten with L in its
    lower and L^T in its upper triangle)."""
    n = int(rhs.shape[0])
    assert V.is_contiguous() and tuple(V.shape) == (n, n)
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=V.device)
    need = int(lib().df3c_fit_solve_workspace(n))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=V.device)
    _check(lib().df3c_fit_solve(_ptr(V), n, _ptr(rhs), _ptr(x), _ptr(ws), ws.numel(), flags,
                                _stream(stream)), "df3c_fit_solve")
    return x


def density_fit(xyz: torch.Tensor, aux: DeviceBasis, orb: DeviceBasis, D: torch.Tensor,
                stream=None) -> torch.Tensor:
    """d = V^{-1} gamma(D): the fitting coefficients of the density D (gamma =
    (P|ab) D, V = (P|Q), Cholesky solve), every step in the library."""
    gamma = coulomb_gamma(xyz, aux, orb, D, stream=stream)
    V = coulomb_metric(xyz, aux, stream=stream)
    return fit_solve(V, gamma, x=gamma, stream=stream)


class CoulombJ(torch.autograd.Function):
    """J(xyz, d) = sum_P (ab|P) d_P as a differentiable function of the atomic
    positions and of the fitting coefficients.  backward(G), G = dL/dJ, runs the
    library's gradient kernel for dL/dxyz and the adjoint digestion
    gamma(G) = sum_ab (P|ab) G_ab for dL/dd."""

    @staticmethod
    def forward(ctx, xyz, d, aux, orb):
        ctx.save_for_backward(xyz, d)
        ctx.aux, ctx.orb = aux, orb
        return coulomb_J(xyz.detach().contiguous(), aux, orb, d.detach().contiguous())

    @staticmethod
    def backward(ctx, gJ):
        xyz, d = ctx.saved_tensors
        G = gJ.detach().to(torch.float64).contiguous()
        gx = gd = None
        if ctx.needs_input_grad[0]:
            gx = coulomb_J_grad(xyz.detach().contiguous(), ctx.aux, ctx.orb,
                                d.detach().contiguous(), G)
        if ctx.needs_input_grad[1]:
            gd = coulomb_gamma(xyz.detach().contiguous(), ctx.aux, ctx.orb, G)
        return gx, gd, None, None


def J(xyz: torch.Tensor, d: torch.Tensor, aux: DeviceBasis, orb: DeviceBasis) -> torch.Tensor:
    """Differentiable DF-J build (see CoulombJ)."""
    return CoulombJ.apply(xyz, d, aux, orb)


def coulomb_J_batched_workspace(aux: DeviceBasis, orb: DeviceBasis, nmol: int,
                                mol_orb: Optional[np.ndarray] = None) -> int:
    """mol_orb is needed for solid-harmonic orbital shells (orb.pure = 1)."""
    sa, so = aux.struct(), orb.struct()
    mo = None if mol_orb is None else np.ascontiguousarray(mol_orb, np.int32)
    return int(lib().df3c_coulomb_J_batched_workspace(ctypes.byref(sa), ctypes.byref(so),
                                                      int(nmol),
                                                      None if mo is None else mo.ctypes.data))


def coulomb_J_batched(xyz: torch.Tensor, aux: DeviceBasis, orb: DeviceBasis,
                      mol_orb: np.ndarray, mol_aux: np.ndarray, d: torch.Tensor,
                      J: Optional[torch.Tensor] = None, tune=None, flags: int = SCHED_PERSISTENT,
                      ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """J of every molecule, concatenated (molecule m's nao_m x nao_m block at
    offset sum_{m'<m} nao_m'^2).  mol_orb / mol_aux: shell ranges per molecule."""
    mol_orb = np.ascontiguousarray(mol_orb, np.int32)
    mol_aux = np.ascontiguousarray(mol_aux, np.int32)
    nmol = len(mol_orb) - 1
    off = orb.offsets()
    nao = off[mol_orb[1:]] - off[mol_orb[:-1]]
    if J is None:
        J = torch.empty(int((nao * nao).sum()), dtype=torch.float64, device=xyz.device)
    need = coulomb_J_batched_workspace(aux, orb, nmol, mol_orb)
    if flags & GRAPH and (ws is None or ws.numel() < need):
        # the cached graph replays against the same workspace address on later
        # calls, so the workspace must be the caller's and outlive them
        raise DF3CError("coulomb_J_batched: GRAPH needs a caller-owned workspace (ws) of "
                        f"at least {need} bytes, kept for every later call")
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=xyz.device)
    sa, so = aux.struct(), orb.struct()
    tp = ctypes.cast(tune, ctypes.c_void_p) if tune is not None else None
    _check(lib().df3c_coulomb_J_batched(_ptr(xyz), int(xyz.shape[0]), ctypes.byref(sa),
                                        ctypes.byref(so), nmol, mol_orb.ctypes.data,
                                        mol_aux.ctypes.data, _ptr(d), _ptr(J), tp, _ptr(ws),
                                        ws.numel(), flags, _stream(stream)),
           "df3c_coulomb_J_batched")
    return J


KERNEL_STORE, KERNEL_J, KERNEL_GRAD, KERNEL_JQ = 0, 1, 2, 3


def timing_enable(on: bool = True) -> None:
    """Bracket every class-kernel launch with HIP events on its stream."""
    _check(lib().df3c_timing_enable(1 if on else 0), "df3c_timing_enable")


def timing_read(cap: int = 65536):
    """Durations of the launches recorded since the last read, as a list of
    (kind, class id, ms); waits for them and clears the record."""
    kind = (ctypes.c_int32 * cap)()
    cls = (ctypes.c_int32 * cap)()
    ms = (ctypes.c_float * cap)()
    n = lib().df3c_timing_read(kind, cls, ms, cap)
    if n < 0:
        _check(int(n), "df3c_timing_read")
    if n > cap:
        raise DF3CError(f"df3c_timing_read: {n} launches recorded, only {cap} could be read")
    return [(int(kind[i]), int(cls[i]), float(ms[i])) for i in range(n)]


def coulomb_J_grad_batched(xyz: torch.Tensor, aux: DeviceBasis, orb: DeviceBasis,
                           mol_orb: np.ndarray, mol_aux: np.ndarray, mol_atom: np.ndarray,
                           d: torch.Tensor, G: torch.Tensor, grad: Optional[torch.Tensor] = None,
                           ws: Optional[torch.Tensor] = None, flags: int = 0,
                           stream=None) -> torch.Tensor:
    """dL/dR [natom][3] of L = sum_m sum_ab G^m_ab J^m_ab over nmol molecules
    (G: the molecules' nao_m x nao_m blocks back to back, as coulomb_J_batched
    returns J)."""
    mol_orb = np.ascontiguousarray(mol_orb, np.int32)
    mol_aux = np.ascontiguousarray(mol_aux, np.int32)
    mol_atom = np.ascontiguousarray(mol_atom, np.int32)
    nmol = len(mol_orb) - 1
    natom = int(xyz.shape[0])
    if grad is None:
        grad = torch.empty((natom, 3), dtype=torch.float64, device=xyz.device)
    sa, so = aux.struct(), orb.struct()
    need = int(lib().df3c_coulomb_J_grad_batched_workspace(
        ctypes.byref(sa), ctypes.byref(so), nmol, mol_orb.ctypes.data, mol_aux.ctypes.data,
        mol_atom.ctypes.data))
    if need == 0:
        raise DF3CError("df3c_coulomb_J_grad_batched_workspace: bad arguments")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=xyz.device)
    _check(lib().df3c_coulomb_J_grad_batched(_ptr(xyz), natom, ctypes.byref(sa), ctypes.byref(so),
                                             nmol, mol_orb.ctypes.data, mol_aux.ctypes.data,
                                             mol_atom.ctypes.data, _ptr(d), _ptr(G.contiguous()),
                                             _ptr(grad), _ptr(ws), ws.numel(), flags,
                                             _stream(stream)), "df3c_coulomb_J_grad_batched")
    return grad
