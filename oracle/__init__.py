"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow McMurchie-Davidson implementation (oracle.c) of the 3-center
Coulomb integrals (P|ab), of J_ab = sum_P (ab|P) d_P, of its adjoint
gamma_P = sum_ab (P|ab) D_ab and of the nuclear gradient of L = sum_ab G_ab J_ab,
wrapped with ctypes.  Only tests/, the smoke check and
the benchmark's CPU-baseline leg may import this package; the GPU library never
does.

Basis arguments are any objects with numpy attributes ``l, nprim, prim_off,
atom, exps, coefs`` and an int attribute ``pure`` (the layout of
``paper_2210_03192_amd.inputs.Basis``).  Coefficients already include all
normalisation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {}


class _Basis(ctypes.Structure):
    _fields_ = [
        ("nshell", ctypes.c_int32),
        ("l", ctypes.c_void_p),
        ("nprim", ctypes.c_void_p),
        ("prim_off", ctypes.c_void_p),
        ("atom", ctypes.c_void_p),
        ("exps", ctypes.c_void_p),
        ("coefs", ctypes.c_void_p),
        ("pure", ctypes.c_int32),
    ]


def _lib(precision="double"):
    name = {"double": "liboracle.so", "long": "liboracle_ld.so"}[precision]
    if name not in _LIBS:
        path = os.path.join(_HERE, name)
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, P]
        lib.oracle_solid_transform.argtypes = [ctypes.c_int, P]
        lib.oracle_eval_batch.argtypes = [P, P, P, ctypes.c_int64, P, P, P, ctypes.c_int]
        lib.oracle_coulomb_J.argtypes = [P, P, P, P, P, ctypes.c_int]
        lib.oracle_coulomb_J_masked.argtypes = [P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_screen_pairs.argtypes = [P, P, ctypes.c_double, P, P]
        lib.oracle_coulomb_gamma.argtypes = [P, P, P, P, P, ctypes.c_int]
        lib.oracle_coulomb_metric.argtypes = [P, P, P, ctypes.c_int]
        lib.oracle_coulomb_J_pairs.argtypes = [P, P, P, P, ctypes.c_int64, P, P, P,
                                               ctypes.c_int]
        lib.oracle_coulomb_J_grad.argtypes = [P, ctypes.c_int32, P, P, P, P, P, P, P,
                                              ctypes.c_int]
        lib.oracle_schwarz_bounds.argtypes = [P, P, P, P, P]
        lib.oracle_screen_pairs_schwarz.argtypes = [P, P, P, P, ctypes.c_double, P, P]
        _LIBS[name] = lib
    return _LIBS[name]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class _Pinned:
    """Holds contiguous copies of a basis' arrays and the C struct over them."""

    def __init__(self, b):
        self.arrs = [np.ascontiguousarray(b.l, np.int32),
                     np.ascontiguousarray(b.nprim, np.int32),
                     np.ascontiguousarray(b.prim_off, np.int64),
                     np.ascontiguousarray(b.atom, np.int32),
                     np.ascontiguousarray(b.exps, np.float64),
                     np.ascontiguousarray(b.coefs, np.float64)]
        self.s = _Basis(len(self.arrs[0]), *[a.ctypes.data for a in self.arrs], int(b.pure))

    @property
    def ref(self):
        return ctypes.byref(self.s)


def ncart(l):
    return (l + 1) * (l + 2) // 2


def nfunc(l, pure):
    return 2 * l + 1 if pure else ncart(l)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (status {rc})")


def boys(mmax, T, precision="double"):
    F = np.zeros(mmax + 1)
    _check(_lib(precision).oracle_boys(int(mmax), float(T), _ptr(F)), "boys")
    return F


def solid_transform(l, precision="double"):
    T = np.zeros((2 * l + 1, ncart(l)))
    _check(_lib(precision).oracle_solid_transform(int(l), _ptr(T)), "solid_transform")
    return T


def eval_batch(xyz, aux, orb, trip, out_off=None, nthreads=0, precision="double"):
    """Blocks (P|ab) for trip[t] = (P, a, b); returns the flat output array and
    the offsets used (dense packing in triplet order if out_off is None)."""
    xyz = np.ascontiguousarray(xyz, np.float64)
    trip = np.ascontiguousarray(trip, np.int32).reshape(-1, 3)
    if len(trip) and (trip.min() < 0 or trip[:, 0].max() >= len(aux.l)
                      or trip[:, 1:].max() >= len(orb.l)):
        raise ValueError("oracle eval_batch: shell index out of range")
    sizes = np.array([nfunc(int(aux.l[p]), aux.pure) * ncart(int(orb.l[a])) * ncart(int(orb.l[b]))
                      for p, a, b in trip], dtype=np.int64)
    if out_off is None:
        out_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if len(sizes) else \
            np.zeros(0, np.int64)
    out_off = np.ascontiguousarray(out_off, np.int64)
    total = int((out_off + sizes).max()) if len(sizes) else 0
    out = np.zeros(total)
    pa, po = _Pinned(aux), _Pinned(orb)
    _check(_lib(precision).oracle_eval_batch(_ptr(xyz), pa.ref, po.ref, len(trip), _ptr(trip),
                                             _ptr(out_off), _ptr(out), int(nthreads)),
           "eval_batch")
    return out, out_off


def coulomb_J(xyz, aux, orb, d, nthreads=0, precision="double"):
    xyz = np.ascontiguousarray(xyz, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    nao = int(sum(nfunc(int(l), orb.pure) for l in orb.l))
    J = np.zeros((nao, nao))
    pa, po = _Pinned(aux), _Pinned(orb)
    _check(_lib(precision).oracle_coulomb_J(_ptr(xyz), pa.ref, po.ref, _ptr(d), _ptr(J),
                                            int(nthreads)), "coulomb_J")
    return J


def coulomb_J_masked(xyz, aux, orb, d, mask, nthreads=0, precision="double"):
    """J over the orbital shell pairs with mask[a, b] != 0 (nshell x nshell,
    symmetric); the other blocks are zero."""
    xyz = np.ascontiguousarray(xyz, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    mask = np.ascontiguousarray(mask, np.uint8)
    assert mask.shape == (len(orb.l), len(orb.l))
    nao = int(sum(ncart(int(l)) for l in orb.l))
    J = np.zeros((nao, nao))
    pa, po = _Pinned(aux), _Pinned(orb)
    _check(_lib(precision).oracle_coulomb_J_masked(_ptr(xyz), pa.ref, po.ref, _ptr(d),
                                                   _ptr(mask), _ptr(J), int(nthreads)),
           "coulomb_J_masked")
    return J


def screen_pairs(xyz, orb, tau):
    """(mask, S): S[a, b] = max_ij |c_ai c_bj| (pi/(z_ai+z_bj))^{3/2}
    exp(-z_ai z_bj/(z_ai+z_bj) |A-B|^2), mask = S >= tau."""
    xyz = np.ascontiguousarray(xyz, np.float64)
    n = len(orb.l)
    mask = np.zeros((n, n), np.uint8)
    S = np.zeros((n, n))
    po = _Pinned(orb)
    _check(_lib().oracle_screen_pairs(_ptr(xyz), po.ref, float(tau), _ptr(mask), _ptr(S)),
           "screen_pairs")
    return mask, S


def coulomb_gamma(xyz, aux, orb, D, nthreads=0, precision="double"):
    """gamma_P = sum_{a,b} (P|ab) D_ab (D: nao x nao, any symmetry)."""
    xyz = np.ascontiguousarray(xyz, np.float64)
    D = np.ascontiguousarray(D, np.float64)
    naux = int(sum(nfunc(int(l), aux.pure) for l in aux.l))
    g = np.zeros(naux)
    pa, po = _Pinned(aux), _Pinned(orb)
    _check(_lib(precision).oracle_coulomb_gamma(_ptr(xyz), pa.ref, po.ref, _ptr(D), _ptr(g),
                                                int(nthreads)), "coulomb_gamma")
    return g


def coulomb_metric(xyz, aux, nthreads=0, precision="double"):
    """V[P][Q] = (P|Q) over the aux basis."""
    xyz = np.ascontiguousarray(xyz, np.float64)
    naux = int(sum(nfunc(int(l), aux.pure) for l in aux.l))
    V = np.zeros((naux, naux))
    pa = _Pinned(aux)
    _check(_lib(precision).oracle_coulomb_metric(_ptr(xyz), pa.ref, _ptr(V), int(nthreads)),
           "coulomb_metric")
    return V


def coulomb_J_pairs(xyz, aux, orb, d, pairs, nthreads=0, precision="double"):
    """List of J blocks (ncart(a) x ncart(b)) for the orbital shell pairs given."""
    xyz = np.ascontiguousarray(xyz, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
    sizes = np.array([ncart(int(orb.l[a])) * ncart(int(orb.l[b])) for a, b in pairs], np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    out = np.zeros(int(sizes.sum()))
    pa, po = _Pinned(aux), _Pinned(orb)
    _check(_lib(precision).oracle_coulomb_J_pairs(_ptr(xyz), pa.ref, po.ref, _ptr(d), len(pairs),
                                                  _ptr(pairs), _ptr(off), _ptr(out),
                                                  int(nthreads)), "coulomb_J_pairs")
    return [out[o:o + s].reshape(ncart(int(orb.l[a])), ncart(int(orb.l[b])))
            for o, s, (a, b) in zip(off, sizes, pairs)]


def coulomb_J_grad(xyz, aux, orb, d, G, atom_mask=None, pair_mask=None, nthreads=0,
                   precision="double"):
    """dL/dR for L = sum_ab G_ab J_ab; with pair_mask (nshell x nshell) J runs
    over the kept shell pairs only."""
    xyz = np.ascontiguousarray(xyz, np.float64)
    natom = xyz.shape[0]
    d = np.ascontiguousarray(d, np.float64)
    G = np.ascontiguousarray(G, np.float64)
    grad = np.zeros((natom, 3))
    mask = None if atom_mask is None else np.ascontiguousarray(atom_mask, np.uint8)
    pm = None if pair_mask is None else np.ascontiguousarray(pair_mask, np.uint8)
    if pm is not None:
        assert pm.shape == (len(orb.l), len(orb.l))
    pa, po = _Pinned(aux), _Pinned(orb)
    _check(_lib(precision).oracle_coulomb_J_grad(_ptr(xyz), natom, pa.ref, po.ref, _ptr(d),
                                                 _ptr(G), None if mask is None else _ptr(mask),
                                                 None if pm is None else _ptr(pm),
                                                 _ptr(grad), int(nthreads)), "coulomb_J_grad")
    return grad


def fit_coefficients(V, gamma):
    """d = V^{-1} gamma, the solution of the density-fitting equations V d =
    gamma (V symmetric positive definite), by its definition: the Cholesky
    factor V = L L^T and the two triangular solves L y = gamma, L^T d = y
    (numpy/scipy routines as the steps)."""
    import scipy.linalg
    V = np.asarray(V, np.float64)
    L = np.linalg.cholesky(V)
    y = scipy.linalg.solve_triangular(L, np.asarray(gamma, np.float64), lower=True)
    return scipy.linalg.solve_triangular(L.T, y, lower=False)


def schwarz_bounds(xyz, aux, orb):
    """(Qab [nshell x nshell], QP [naux shells]) with |(ab|P_m)| <= Qab QP."""
    xyz = np.ascontiguousarray(xyz, np.float64)
    n = len(orb.l)
    Qab = np.zeros((n, n))
    QP = np.zeros(len(aux.l))
    pa, po = _Pinned(aux), _Pinned(orb)
    _check(_lib().oracle_schwarz_bounds(_ptr(xyz), pa.ref, po.ref, _ptr(Qab), _ptr(QP)),
           "schwarz_bounds")
    return Qab, QP


def screen_pairs_schwarz(xyz, aux, orb, d, tau):
    """(mask, S_d): mask = Qab S_d >= tau, S_d = sum_P QP sum_m |d_Pm|."""
    xyz = np.ascontiguousarray(xyz, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    n = len(orb.l)
    mask = np.zeros((n, n), np.uint8)
    Sd = np.zeros(1)
    pa, po = _Pinned(aux), _Pinned(orb)
    _check(_lib().oracle_screen_pairs_schwarz(_ptr(xyz), pa.ref, po.ref, _ptr(d), float(tau),
                                              _ptr(mask), _ptr(Sd)), "screen_pairs_schwarz")
    return mask, float(Sd[0])
