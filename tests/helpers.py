"""Small builders shared by the tests (no integral arithmetic)."""
import numpy as np

from paper_2210_03192_amd.inputs import Basis, ncart, npure


def single_triplet(A, B, C, la, lb, lc, za, zb, zc, ca=None, cb=None, cc=None, pure=0):
    """One triplet (P at C, a at A, b at B).  Exponent arguments may be lists
    (contracted shells); coefficients default to 1 (unnormalised primitives)."""
    za, zb, zc = (np.atleast_1d(np.asarray(z, float)) for z in (za, zb, zc))
    ca = np.ones_like(za) if ca is None else np.atleast_1d(np.asarray(ca, float))
    cb = np.ones_like(zb) if cb is None else np.atleast_1d(np.asarray(cb, float))
    cc = np.ones_like(zc) if cc is None else np.atleast_1d(np.asarray(cc, float))
    xyz = np.array([C, A, B], float)
    aux = Basis(np.array([lc], np.int32), np.array([len(zc)], np.int32), np.array([0], np.int64),
                np.array([0], np.int32), zc, cc, pure)
    orb = Basis(np.array([la, lb], np.int32), np.array([len(za), len(zb)], np.int32),
                np.array([0, len(za)], np.int64), np.array([1, 2], np.int32),
                np.concatenate([za, zb]), np.concatenate([ca, cb]), 0)
    trip = np.array([[0, 0, 1]], np.int32)
    return xyz, aux, orb, trip


def block_shape(lc, la, lb, pure):
    return (npure(lc) if pure else ncart(lc), ncart(la), ncart(lb))


def close_shell_pairs(orb, xyz, seed, per_class=3, max_dist=3.0):
    """Orbital shell pairs (a, b) whose centres lie within max_dist bohr of each
    other (same atom or a bonded neighbour), per_class of them for every
    (l_a >= l_b) combination the basis has, drawn with a seeded generator.
    Their J blocks are the largest of a molecule, so the relative part of the
    parity bar applies to most of their elements."""
    rng = np.random.default_rng(seed)
    l = np.asarray(orb.l)
    atom = np.asarray(orb.atom)
    dist = np.sqrt(((xyz[atom][:, None, :] - xyz[atom][None, :, :]) ** 2).sum(-1))
    pairs = []
    for la in range(int(l.max()) + 1):
        for lb in range(la + 1):
            a_idx, b_idx = np.nonzero((l[:, None] == la) & (l[None, :] == lb) & (dist <= max_dist))
            if not len(a_idx):
                continue
            pick = rng.choice(len(a_idx), min(per_class, len(a_idx)), replace=False)
            pairs += [(int(a_idx[k]), int(b_idx[k])) for k in pick]
    return np.array(pairs, np.int32).reshape(-1, 2)
