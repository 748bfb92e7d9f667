"""Parity bars of gamma_P = sum_ab (P|ab) D_ab and J_ab = sum_P (ab|P) d_P.

gamma sums many terms of both signs, so its elements can be far smaller than
the terms.  Each term is an integral held to max(1e-11 |x|, 1e-13) times a
fixed D_ab; the bar of a gamma element is the sum of its terms' bars,
    B_P = sum_ab |D_ab| max(1e-11 |(P|ab)|, 1e-13),
with the oracle's blocks (the bar of J carried through a linear map, as for
the solid-harmonic J).  With solid-harmonic orbital shells D acts through
the transform, D_cart = T_a^T D T_b, and |D| is carried as |T_a|^T |D| |T_b|.
"""
import numpy as np

import oracle


def _cart_abs(orb, D):
    """|D| over Cartesian orbital components (carried through |T| for pure)."""
    if not orb.pure:
        return np.abs(D)
    from paper_2210_03192_amd.inputs import Basis
    cart = Basis(orb.l, orb.nprim, orb.prim_off, orb.atom, orb.exps, orb.coefs, pure=0)
    oc, op = cart.offsets(), orb.offsets()
    T = [np.abs(oracle.solid_transform(int(l))) for l in orb.l]
    out = np.zeros((oc[-1], oc[-1]))
    for a in range(orb.nshell):
        for b in range(orb.nshell):
            out[oc[a]:oc[a + 1], oc[b]:oc[b + 1]] = \
                T[a].T @ np.abs(D[op[a]:op[a + 1], op[b]:op[b + 1]]) @ T[b]
    return out


def gamma_bar(xyz, aux, orb, D):
    from paper_2210_03192_amd.inputs import Basis, ncart
    cart = Basis(orb.l, orb.nprim, orb.prim_off, orb.atom, orb.exps, orb.coefs, pure=0)
    Dabs = _cart_abs(orb, D)
    trip = np.array([(P, a, b) for P in range(aux.nshell) for a in range(orb.nshell)
                     for b in range(orb.nshell)], np.int32)
    blocks, off = oracle.eval_batch(xyz, aux, cart, trip)
    ao, po = cart.offsets(), aux.offsets()
    bar = np.zeros(int(po[-1]))
    for (P, a, b), o in zip(trip, off):
        nP, na, nb = aux.nfunc(P), ncart(int(orb.l[a])), ncart(int(orb.l[b]))
        blk = np.abs(blocks[o:o + nP * na * nb].reshape(nP, na, nb))
        bar[po[P]:po[P + 1]] += np.einsum("pab,ab->p", np.maximum(1e-11 * blk, 1e-13),
                                          Dabs[ao[a]:ao[a + 1], ao[b]:ao[b + 1]])
    return bar


def assert_gamma(g, xyz, aux, orb, D, what):
    """gamma against the oracle at the element bar max(1e-11 |ref|, 1e-13);
    elements outside are adjudicated by the long-double oracle.  The carried
    bar B_P is reported beside it."""
    ref = oracle.coulomb_gamma(xyz, aux, orb, D)

    def bad(r):
        return np.abs(g - r) > np.maximum(1e-11 * np.abs(r), 1e-13)
    if bad(ref).any():
        ref = oracle.coulomb_gamma(xyz, aux, orb, D, precision="long")
    b = bad(ref)
    assert not b.any(), (what, int(b.sum()), float(np.abs(g - ref).max()))
    bar = gamma_bar(xyz, aux, orb, D)
    plain = np.maximum(1e-11 * np.abs(ref), 1e-13)
    print(f"{what}: max |err|/element bar {float((np.abs(g - ref) / plain).max()):.3g}, "
          f"max |err|/carried bar {float((np.abs(g - ref) / bar).max()):.3g}")


def j_pair_bars(xyz, aux, orb, d, pairs):
    """The same carried bar for J blocks of Cartesian orbital shell pairs:
    B_ab = sum_P |d_P| max(1e-11 |(ab|P)|, 1e-13), from the oracle's blocks
    of every aux shell with the pair.  J_ab is a sum over the fitting
    functions as gamma_P is over the pairs."""
    from paper_2210_03192_amd.inputs import ncart
    po = aux.offsets()
    out = []
    for a, b in pairs:
        trip = np.array([(P, a, b) for P in range(aux.nshell)], np.int32)
        blocks, off = oracle.eval_batch(xyz, aux, orb, trip)
        na, nb = ncart(int(orb.l[a])), ncart(int(orb.l[b]))
        bar = np.zeros((na, nb))
        for (P, _, _), o in zip(trip, off):
            nP = aux.nfunc(P)
            blk = np.abs(blocks[o:o + nP * na * nb].reshape(nP, na, nb))
            bar += np.einsum("pab,p->ab", np.maximum(1e-11 * blk, 1e-13),
                             np.abs(d[po[P]:po[P + 1]]))
        out.append(bar)
    return out
