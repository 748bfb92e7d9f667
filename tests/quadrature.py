"""Brute-force numerical quadrature of primitive 3-center Coulomb integrals.

Test helper only.  It shares no formula with the McMurchie-Davidson oracle, the
Boys function or the Obara-Saika recurrences:

  1/r12 = (2/sqrt(pi)) int_0^inf exp(-t^2 r12^2) dt,

and for fixed t the 6-D integral over r1, r2 factorises into one 2-D integral
per Cartesian axis, a polynomial times a 2-D Gaussian.  That 2-D integral is
evaluated exactly by tensor Gauss-Hermite quadrature after the affine map that
takes the Gaussian to exp(-|y|^2); the outer t integral uses scipy's adaptive
vector quadrature.
"""
import numpy as np
from scipy.integrate import quad_vec

GH_Y, GH_W = np.polynomial.hermite.hermgauss(12)


def carts(l):
    return [(l - i, i - j, j) for i in range(l + 1) for j in range(i + 1)]


def _axis_table(A, B, C, la, lb, lc, za, zb, zc, t):
    """I[ax][bx][cx] = int int (x1-A)^ax (x1-B)^bx (x2-C)^cx
       exp(-za (x1-A)^2 - zb (x1-B)^2 - t^2 (x1-x2)^2 - zc (x2-C)^2) dx1 dx2."""
    t2 = t * t
    a, c = za + zb, zc
    h = np.array([za * A + zb * B, zc * C])
    det = t2 * (a + c) + a * c
    mu = np.array([(t2 + c) * h[0] + t2 * h[1], t2 * h[0] + (a + t2) * h[1]]) / det
    kk = za * A * A + zb * B * B + zc * C * C
    const = np.exp(-(kk - h @ mu))
    # Cholesky of M = [[a+t2, -t2], [-t2, t2+c]] without cancellation
    L11 = np.sqrt(a + t2)
    L21 = -t2 / L11
    L22 = np.sqrt(det / (a + t2))
    # x = mu + L^{-T} y;  L^{-T} = [[1/L11, -L21/(L11 L22)], [0, 1/L22]]
    y1, y2 = np.meshgrid(GH_Y, GH_Y, indexing="ij")
    w = np.outer(GH_W, GH_W)
    x1 = mu[0] + y1 / L11 - L21 / (L11 * L22) * y2
    x2 = mu[1] + y2 / L22
    jac = 1.0 / (L11 * L22)
    pa = np.stack([(x1 - A) ** k for k in range(la + 1)])
    pb = np.stack([(x1 - B) ** k for k in range(lb + 1)])
    pc = np.stack([(x2 - C) ** k for k in range(lc + 1)])
    return const * jac * np.einsum("aij,bij,cij,ij->abc", pa, pb, pc, w)


def primitive_block(A, B, C, la, lb, lc, za, zb, zc, epsrel=1e-13):
    """[c][a][b] Cartesian block of primitive integrals (coefficients 1)."""
    A, B, C = (np.asarray(v, float) for v in (A, B, C))
    shift = (A + B + C) / 3
    A, B, C = A - shift, B - shift, C - shift
    qa, qb, qc = carts(la), carts(lb), carts(lc)
    ia = np.array(qa)
    ib = np.array(qb)
    ic = np.array(qc)

    def f(t):
        tabs = [_axis_table(A[k], B[k], C[k], la, lb, lc, za, zb, zc, t) for k in range(3)]
        out = np.ones((len(qc), len(qa), len(qb)))
        for k in range(3):
            out *= tabs[k][ia[None, :, None, k], ib[None, None, :, k], ic[:, None, None, k]]
        return out * (2 / np.sqrt(np.pi))

    val, err = quad_vec(f, 0, np.inf, epsrel=epsrel, epsabs=0, limit=4000)
    return val
