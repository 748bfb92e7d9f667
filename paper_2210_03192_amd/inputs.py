"""Seeded synthetic inputs shared by the GPU library's tests/benchmark and the
CPU oracle's tests.  This module holds no integral arithmetic: it builds
geometries, basis-set descriptors (angular momenta, exponents, normalised
contraction coefficients), triplet lists and random fitting coefficients.

Basis-set conventions:
  * a shell is a set of Cartesian Gaussians with l quanta (Appendix "Notation");
  * contraction coefficients include the primitive normalisation
    N(zeta, l) = (2 zeta/pi)^{3/4} (4 zeta)^{l/2} / sqrt((2l-1)!!) of the x^l
    component, rescaled so the contracted x^l component has unit self-overlap;
  * orbital shells are Cartesian (pure = 0), auxiliary shells solid-harmonic
    (pure = 1), the ket form of Section 2.2.
"""
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 20221003


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def npure(l: int) -> int:
    return 2 * l + 1


@dataclass
class Basis:
    l: np.ndarray          # int32 [nshell]
    nprim: np.ndarray      # int32 [nshell]
    prim_off: np.ndarray   # int64 [nshell]
    atom: np.ndarray       # int32 [nshell]
    exps: np.ndarray       # float64 [nprim_total]
    coefs: np.ndarray      # float64 [nprim_total]
    pure: int = 0

    @property
    def nshell(self) -> int:
        return int(len(self.l))

    def nfunc(self, s: int) -> int:
        l = int(self.l[s])
        return npure(l) if self.pure else ncart(l)

    def offsets(self) -> np.ndarray:
        """Function offset of every shell, plus the total at the end."""
        n = np.array([npure(int(l)) if self.pure else ncart(int(l)) for l in self.l], np.int64)
        return np.concatenate([[0], np.cumsum(n)]).astype(np.int64)

    @property
    def nbf(self) -> int:
        return int(self.offsets()[-1])


@dataclass
class System:
    """One molecule: atom positions (bohr), orbital and auxiliary bases."""
    xyz: np.ndarray        # float64 [natom, 3]
    orb: Basis
    aux: Basis
    name: str = ""


def _dfact(n: int) -> float:
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


def normalise(l: int, exps: Sequence[float], coefs: Sequence[float]) -> np.ndarray:
    """Coefficients with primitive normalisation folded in and the contracted
    x^l component scaled to unit self-overlap."""
    e = np.asarray(exps, np.float64)
    c = np.asarray(coefs, np.float64)
    N = (2 * e / np.pi) ** 0.75 * (4 * e) ** (l / 2) / np.sqrt(_dfact(2 * l - 1))
    S = (2 * np.sqrt(np.outer(e, e)) / np.add.outer(e, e)) ** (l + 1.5)
    s = float(c @ S @ c)
    return c * N / np.sqrt(s)


class _Builder:
    def __init__(self, pure: int):
        self.pure = pure
        self.l: List[int] = []
        self.nprim: List[int] = []
        self.atom: List[int] = []
        self.exps: List[float] = []
        self.coefs: List[float] = []

    def add(self, l: int, atom: int, exps, coefs):
        self.l.append(l)
        self.nprim.append(len(exps))
        self.atom.append(atom)
        self.exps.extend(float(x) for x in exps)
        self.coefs.extend(float(x) for x in normalise(l, exps, coefs))

    def build(self) -> Basis:
        nprim = np.array(self.nprim, np.int32)
        off = np.concatenate([[0], np.cumsum(nprim)[:-1]]).astype(np.int64) if len(nprim) \
            else np.zeros(0, np.int64)
        return Basis(np.array(self.l, np.int32), nprim, off, np.array(self.atom, np.int32),
                     np.array(self.exps, np.float64), np.array(self.coefs, np.float64),
                     self.pure)


def _logu(rng, lo, hi, n):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def random_atoms(rng, n: int, box: float, min_sep: float) -> np.ndarray:
    """n points uniform in [0, box]^3, redrawn until every pair is >= min_sep apart."""
    while True:
        x = rng.uniform(0, box, (n, 3))
        d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
        d[np.arange(n), np.arange(n)] = np.inf
        if d.min() >= min_sep:
            return x


# --------------------------------------------------------------------------
# Plain DF-J system: 8 atoms in a 6 bohr cube
# --------------------------------------------------------------------------
def plain_dfj_system(seed: int = SEED_BASE + 1, natom: int = 8) -> System:
    """Atoms uniform in [0,6]^3 bohr (pairs >= 1.5 bohr apart).  Orbital shells
    per atom: s, s, p, d with K = 3 (exponents log-uniform in [0.1, 50],
    coefficients uniform in [0.1, 1]); auxiliary shells 4s3p2d1f uncontracted
    (exponents log-uniform in [0.05, 20]).  Independent draws per atom."""
    rng = np.random.default_rng(seed)
    xyz = random_atoms(rng, natom, 6.0, 1.5)
    ob, ab = _Builder(0), _Builder(1)
    for a in range(natom):
        for l in (0, 0, 1, 2):
            ob.add(l, a, _logu(rng, 0.1, 50.0, 3), rng.uniform(0.1, 1.0, 3))
        for l, n in ((0, 4), (1, 3), (2, 2), (3, 1)):
            for _ in range(n):
                ab.add(l, a, _logu(rng, 0.05, 20.0, 1), [1.0])
    return System(xyz, ob.build(), ab.build(), "plain-dfj-8atoms")


# --------------------------------------------------------------------------
# Per-class batches: fresh random centres per triplet
# --------------------------------------------------------------------------
@dataclass
class ClassBatch:
    LP: int
    la: int
    lb: int
    K: int                 # contraction degree of a and of b (K_P = 1)
    xyz: np.ndarray
    aux: Basis
    orb: Basis
    trip: np.ndarray       # int32 [ntrip, 3] = (P, a, b)
    out_off: np.ndarray    # int64 [ntrip]
    block: int             # doubles per block

    @property
    def ntrip(self) -> int:
        return int(len(self.trip))

    @property
    def nint(self) -> int:
        return self.ntrip * self.block


def class_batch(LP: int, la: int, lb: int, K: int, ntrip: int, seed: Optional[int] = None,
                box: float = 20.0, zlo: float = 0.05, zhi: float = 100.0) -> ClassBatch:
    """ntrip triplets of one class (L_P, l_a, l_b); each triplet has three fresh
    centres uniform in a box, exponents log-uniform in [zlo, zhi], coefficients
    uniform in [0.1, 1] (normalised).  Output blocks are packed densely."""
    if seed is None:
        seed = SEED_BASE + 2 + 1000 * LP + 100 * la + 10 * lb + K
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(0, box, (3 * ntrip, 3))
    # vectorised shell construction (the builder loop is slow at 1e5 triplets)
    ea = _logu(rng, zlo, zhi, ntrip * K).reshape(ntrip, K)
    eb = _logu(rng, zlo, zhi, ntrip * K).reshape(ntrip, K)
    ec = _logu(rng, zlo, zhi, ntrip).reshape(ntrip, 1)
    ca = rng.uniform(0.1, 1.0, (ntrip, K))
    cb = rng.uniform(0.1, 1.0, (ntrip, K))
    cc = np.ones((ntrip, 1))

    def norm_rows(l, e, c):
        N = (2 * e / np.pi) ** 0.75 * (4 * e) ** (l / 2) / np.sqrt(_dfact(2 * l - 1))
        S = (2 * np.sqrt(e[:, :, None] * e[:, None, :]) / (e[:, :, None] + e[:, None, :])) \
            ** (l + 1.5)
        s = np.einsum("ti,tij,tj->t", c, S, c)
        return c * N / np.sqrt(s)[:, None]

    ca, cb, cc = norm_rows(la, ea, ca), norm_rows(lb, eb, cb), norm_rows(LP, ec, cc)
    aux = Basis(np.full(ntrip, LP, np.int32), np.ones(ntrip, np.int32),
                np.arange(ntrip, dtype=np.int64), (3 * np.arange(ntrip)).astype(np.int32),
                ec.ravel().copy(), cc.ravel().copy(), 1)
    # orbital shells interleaved: shell 2t = a (atom 3t+1), 2t+1 = b (atom 3t+2)
    l = np.empty(2 * ntrip, np.int32)
    l[0::2], l[1::2] = la, lb
    e = np.empty((2 * ntrip, K))
    e[0::2], e[1::2] = ea, eb
    c = np.empty((2 * ntrip, K))
    c[0::2], c[1::2] = ca, cb
    atom = np.empty(2 * ntrip, np.int32)
    atom[0::2] = 3 * np.arange(ntrip) + 1
    atom[1::2] = 3 * np.arange(ntrip) + 2
    orb = Basis(l, np.full(2 * ntrip, K, np.int32), (K * np.arange(2 * ntrip)).astype(np.int64),
                atom, e.ravel().copy(), c.ravel().copy(), 0)
    trip = np.stack([np.arange(ntrip), 2 * np.arange(ntrip), 2 * np.arange(ntrip) + 1],
                    1).astype(np.int32)
    block = npure(LP) * ncart(la) * ncart(lb)
    out_off = (block * np.arange(ntrip)).astype(np.int64)
    return ClassBatch(LP, la, lb, K, xyz, aux, orb, trip, out_off, block)


PER_CLASS_CLASSES: Tuple[Tuple[int, int, int], ...] = (
    (0, 0, 0), (2, 1, 1), (4, 2, 2), (6, 3, 3), (6, 4, 4))
PER_CLASS_K: Tuple[int, ...] = (1, 3, 6)


# --------------------------------------------------------------------------
# Water clusters
# --------------------------------------------------------------------------
R_OH = 1.81
ANGLE_HOH = np.deg2rad(104.5)
# (l, K) of every orbital shell; auxiliary shells are uncontracted
ORB_SHELLS = {
    "O": [(0, 6), (0, 3), (0, 1), (0, 1), (1, 3), (1, 1), (1, 1), (2, 1), (2, 1), (3, 1)],
    "H": [(0, 3), (0, 1), (0, 1), (1, 1), (1, 1), (2, 1)],
}
AUX_SHELLS = {
    "O": [0] * 8 + [1] * 7 + [2] * 6 + [3] * 4 + [4] * 3 + [5] * 2 + [6] * 1,
    "H": [0] * 5 + [1] * 4 + [2] * 3 + [3] * 2 + [4] * 1,
}


def element_basis(seed: int = SEED_BASE + 100):
    """Exponents and raw coefficients drawn once per element: orbital exponents
    log-uniform in [0.1, 50], auxiliary in [0.05, 20], coefficients U[0.1, 1]."""
    rng = np.random.default_rng(seed)
    out = {}
    for el in ("O", "H"):
        orb = [(l, _logu(rng, 0.1, 50.0, K), rng.uniform(0.1, 1.0, K)) for l, K in ORB_SHELLS[el]]
        aux = [(l, _logu(rng, 0.05, 20.0, 1), np.ones(1)) for l in AUX_SHELLS[el]]
        out[el] = (orb, aux)
    return out


def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def water_geometry(n_w: int, rng) -> Tuple[np.ndarray, List[str]]:
    """n_w waters (O-H 1.81 bohr, H-O-H 104.5 deg, random orientations) inserted
    sequentially at random points of a sphere of radius (225 n_w / pi)^(1/3)
    bohr, keeping every O-O distance >= 5 bohr."""
    R = (225.0 * n_w / np.pi) ** (1.0 / 3.0)
    h = ANGLE_HOH / 2
    local = np.array([[0, 0, 0], [R_OH * np.sin(h), 0, R_OH * np.cos(h)],
                      [-R_OH * np.sin(h), 0, R_OH * np.cos(h)]])
    oxy: List[np.ndarray] = []
    xyz, els = [], []
    while len(oxy) < n_w:
        p = rng.uniform(-R, R, 3)
        if np.linalg.norm(p) > R:
            continue
        if oxy and np.min(np.linalg.norm(np.array(oxy) - p, axis=1)) < 5.0:
            continue
        oxy.append(p)
        xyz.append(local @ _random_rotation(rng).T + p)
        els += ["O", "H", "H"]
    return np.concatenate(xyz, 0), els


def water_cluster(n_w: int, seed: int, basis_seed: int = SEED_BASE + 100) -> System:
    rng = np.random.default_rng(seed)
    xyz, els = water_geometry(n_w, rng)
    eb = element_basis(basis_seed)
    ob, ab = _Builder(0), _Builder(1)
    for a, el in enumerate(els):
        orb, aux = eb[el]
        for l, e, c in orb:
            ob.add(l, a, e, c)
        for l, e, c in aux:
            ab.add(l, a, e, c)
    return System(xyz, ob.build(), ab.build(), f"water{n_w}")


def dfj_120_system(seed: int = SEED_BASE + 3) -> System:
    """40 waters (120 atoms)."""
    return water_cluster(40, seed)


def grad_60_system(seed: int = SEED_BASE + 5) -> System:
    """20 waters (60 atoms)."""
    return water_cluster(20, seed)


def batched_systems(nmol: int = 64, seed: int = SEED_BASE + 4, lo: int = 5, hi: int = 50) \
        -> List[System]:
    """nmol clusters with n_w ~ U{lo..hi} waters (15..150 atoms)."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, nmol)
    return [water_cluster(int(n), seed * 1000 + i) for i, n in enumerate(sizes)]


def fitting_coefficients(naux: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).normal(size=naux)


def symmetric_density(nao: int, seed: int) -> np.ndarray:
    X = np.random.default_rng(seed).normal(size=(nao, nao))
    return (X + X.T) / 2


@dataclass
class Batch:
    """Several molecules in one system: shells of molecule m are
    orb[mol_orb[m]:mol_orb[m+1]] and aux[mol_aux[m]:mol_aux[m+1]]."""
    xyz: np.ndarray
    orb: Basis
    aux: Basis
    mol_orb: np.ndarray
    mol_aux: np.ndarray
    systems: List[System]

    @property
    def nmol(self) -> int:
        return len(self.systems)


def _concat_basis(parts: List[Basis], atom_off: List[int]) -> Basis:
    prim = 0
    l, nprim, off, atom, exps, coefs = [], [], [], [], [], []
    for b, ao in zip(parts, atom_off):
        l.append(b.l)
        nprim.append(b.nprim)
        off.append(b.prim_off + prim)
        atom.append(b.atom + ao)
        exps.append(b.exps)
        coefs.append(b.coefs)
        prim += len(b.exps)
    return Basis(np.concatenate(l).astype(np.int32), np.concatenate(nprim).astype(np.int32),
                 np.concatenate(off).astype(np.int64), np.concatenate(atom).astype(np.int32),
                 np.concatenate(exps), np.concatenate(coefs), parts[0].pure)


def concat_systems(systems: List[System]) -> Batch:
    atom_off = list(np.cumsum([0] + [len(s.xyz) for s in systems[:-1]]))
    orb = _concat_basis([s.orb for s in systems], atom_off)
    aux = _concat_basis([s.aux for s in systems], atom_off)
    mol_orb = np.concatenate([[0], np.cumsum([s.orb.nshell for s in systems])]).astype(np.int32)
    mol_aux = np.concatenate([[0], np.cumsum([s.aux.nshell for s in systems])]).astype(np.int32)
    return Batch(np.concatenate([s.xyz for s in systems]), orb, aux, mol_orb, mol_aux, systems)
