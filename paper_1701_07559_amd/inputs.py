"""Seeded synthetic inputs for the Moebius domain-wall solve.

This module holds only input generation: gauge links, 5D sources, random
gauge transforms, and the plaquette that characterises a generated field.  It
contains none of the Dirac-operator arithmetic, so the CPU oracle and the HIP
path can both consume its output without sharing any of the method.

Conventions (host canonical layouts, all complex128):

* gauge field ``U[t, z, y, x, mu, a, b]`` -- the SU(3) link ``U_mu(x)`` with
  row ``a`` and column ``b``; ``mu`` = 0..3 for x, y, z, t.
* 5D spinor ``psi[s, t, z, y, x, spin, colour]`` with 4 spins and 3 colours;
  spins 0,1 are the positive-chirality (upper) components and 2,3 the
  negative-chirality (lower) ones in the chiral gamma basis.

The paper's valence action lives on smoothed (gradient-flowed) HISQ gauge
ensembles (Sec. II, Table I).  Those ensembles are not available here, so a
smooth random SU(3) field ``U = exp(i eps H)`` stands in for them, with the
ensembles' lattice shapes.  ``H`` is a traceless Hermitian Gaussian matrix
normalised so that E tr H^2 = 10; at eps = 0.25 the average plaquette is about
0.65.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "random_links",
    "unit_links",
    "gaussian_source",
    "point_source",
    "point_source_columns",
    "random_gauge_transform",
    "gauge_transform_links",
    "gauge_transform_spinor",
    "plaquette",
    "random_point_site",
]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3), tr(l_a l_b) = 2 delta_ab."""
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0][0, 1] = g[0][1, 0] = 1
    g[1][0, 1], g[1][1, 0] = -1j, 1j
    g[2][0, 0], g[2][1, 1] = 1, -1
    g[3][0, 2] = g[3][2, 0] = 1
    g[4][0, 2], g[4][2, 0] = -1j, 1j
    g[5][1, 2] = g[5][2, 1] = 1
    g[6][1, 2], g[6][2, 1] = -1j, 1j
    g[7][0, 0] = g[7][1, 1] = 1 / np.sqrt(3)
    g[7][2, 2] = -2 / np.sqrt(3)
    return g


def _rng(seed: int) -> np.random.Generator:
    # Philox4x64 counter-based generator; its stream is fixed for a seed.
    return np.random.Generator(np.random.Philox(key=int(seed)))


def _exp_iH(H: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for a stack of Hermitian 3x3 matrices, via eigh."""
    w, v = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ab,...b,...cb->...ac", v, ph, v.conj())


def _links_slice(h: np.ndarray, lam: np.ndarray, eps: float) -> np.ndarray:
    return _exp_iH(np.tensordot(h, lam, axes=([4], [0])), eps)


def random_links(dims, eps: float, seed: int, workers: int = 1) -> np.ndarray:
    """Smooth random SU(3) links ``U = exp(i eps H)``, i.i.d. per link.

    ``dims`` = (X, Y, Z, T).  ``H = sqrt(5/8) sum_a h_a lambda_a`` with
    h_a ~ N(0, 1).  Generated one time-slice at a time so that memory stays
    bounded at the largest shapes; the stream order does not depend on that.
    ``workers`` > 1 draws the normals in the same order in this process and
    exponentiates the slices in forked worker processes (bitwise the same
    field); call it before the process has touched a GPU.
    """
    X, Y, Z, T = (int(d) for d in dims)
    lam = gell_mann() * np.sqrt(5.0 / 8.0)
    rng = _rng(seed)
    U = np.empty((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    if workers <= 1 or T < 2:
        for t in range(T):
            U[t] = _links_slice(rng.standard_normal((Z, Y, X, 4, 8)), lam, eps)
        return U
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(int(workers), mp_context=mp.get_context("fork")) as ex:
        futs = [ex.submit(_links_slice, rng.standard_normal((Z, Y, X, 4, 8)), lam, eps) for _ in range(T)]
        for t, f in enumerate(futs):
            U[t] = f.result()
    return U


def unit_links(dims) -> np.ndarray:
    X, Y, Z, T = (int(d) for d in dims)
    U = np.zeros((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def gaussian_source(dims, L5: int, seed: int) -> np.ndarray:
    """Full 5D source with Re and Im of every component i.i.d. N(0, 1)."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = _rng(seed)
    shape = (int(L5), T, Z, Y, X, 4, 3)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


def random_point_site(dims, seed: int):
    """A seeded lattice site (x, y, z, t)."""
    rng = _rng(seed)
    return tuple(int(rng.integers(0, d)) for d in dims)


def point_source(dims, L5: int, site, spin: int, colour: int) -> np.ndarray:
    """5D right-hand side for a 4D point source.

    The 4D source eta is a unit vector at ``site`` with the given spin and
    colour.  Its negative-chirality part enters on the first slice and its
    positive-chirality part on the last slice, the usual domain-wall wall
    assignment: b[0] = P_- eta, b[L5-1] = P_+ eta.
    """
    X, Y, Z, T = (int(d) for d in dims)
    x, y, z, t = site
    b = np.zeros((int(L5), T, Z, Y, X, 4, 3), dtype=np.complex128)
    s = int(L5) - 1 if spin < 2 else 0
    b[s, t, z, y, x, spin, colour] = 1.0
    return b


def point_source_columns(dims, L5: int, site):
    """The 12 spin-colour columns of a point source, in order spin*3+colour."""
    return [point_source(dims, L5, site, sp, c) for sp in range(4) for c in range(3)]


def _haar_su3(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random SU(3) matrices via QR of a complex Ginibre matrix.

    The phases of R's diagonal are moved into Q so that Q is Haar on U(3)
    (Mezzadri, Notices AMS 54 (2007) 592); dividing by a cube root of the
    determinant then lands in SU(3).
    """
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return q


def random_gauge_transform(dims, seed: int) -> np.ndarray:
    """g[t, z, y, x, a, b]: one Haar-random SU(3) matrix per site."""
    X, Y, Z, T = (int(d) for d in dims)
    g = _haar_su3(X * Y * Z * T, _rng(seed))
    return g.reshape(T, Z, Y, X, 3, 3)


def _shift(a: np.ndarray, mu: int, k: int = 1) -> np.ndarray:
    """a(x + k mu-hat) with periodic wrap; axes are (t, z, y, x, ...)."""
    axis = 3 - mu
    return np.roll(a, -k, axis=axis)


def gauge_transform_links(U: np.ndarray, g: np.ndarray) -> np.ndarray:
    """U_mu(x) -> g(x) U_mu(x) g(x + mu)^dagger."""
    out = np.empty_like(U)
    for mu in range(4):
        gp = _shift(g, mu)
        out[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gp, -1, -2))
    return out


def gauge_transform_spinor(psi: np.ndarray, g: np.ndarray) -> np.ndarray:
    """psi(x, s) -> g(x) psi(x, s), acting on colour."""
    return np.einsum("tzyxab,...tzyxsb->...tzyxsa", g, psi)


def plaquette(U: np.ndarray) -> float:
    """Average plaquette (1/3) Re tr U_mu U_nu(x+mu) U_mu(x+nu)^+ U_nu^+.

    Averaged over all sites and the six planes; describes how smooth a
    generated field is (the paper lists flowed plaquettes in its tables).
    """
    tot = 0.0
    n = 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Um = U[..., mu, :, :]
            Un = U[..., nu, :, :]
            Un_xm = _shift(Un, mu)
            Um_xn = _shift(Um, nu)
            loop = Um @ Un_xm @ np.conj(np.swapaxes(Um_xn, -1, -2)) @ np.conj(np.swapaxes(Un, -1, -2))
            tot += np.trace(loop, axis1=-2, axis2=-1).real.mean() / 3.0
            n += 1
    return tot / n
