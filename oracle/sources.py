"""Source and sink side of the propagator solve -- FP64 CPU reference.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU baseline of
the benchmark use this module; the library never does.  It shares no code
with the HIP path (the Wilson operator D_W comes from the C oracle).

What is computed:

* Gauge-covariant Gaussian smearing of a 4D source (the paper's MDWF
  propagators are solved from such sources, Sec. V, citing Frommer et al.):
      psi <- (1 + sigma^2 / (4 N) Delta)^N psi,
      (Delta psi)(x) = sum_{i = x, y, z} [U_i(x) psi(x + i) + U_i(x - i)^+ psi(x - i) - 2 psi(x)],
  applied within each time slice, spin and colour structure untouched
  except for the links' colour rotation; spatial directions periodic.

* The 5D right-hand side whose solution carries the physical 4D quark
  propagator, for D5 = D_W B + 1 - C with (C psi)_s = P- psi_{s+1} + P+ psi_{s-1}
  (wrap -m_q):
      b = (1 - c5 D_W) Pbar eta,   (Pbar eta)_{L5-1} = P- eta,  (Pbar eta)_0 = P+ eta,
  i.e. the source of the wall antiquark qbar = psibar_{L5-1} P- + psibar_0 P+,
  with the factor (1 - c5 D_W) that the Moebius coupling of neighbouring
  slices puts on it (c5 = 0: the Shamir source).

* The wall and midpoint 4D fields of a 5D solution x (Sec. III, m_res):
      q(x) = P- x_0 + P+ x_{L5-1},          Q(x) = P- x_{L5/2} + P+ x_{L5/2-1},
  and, from the 12 spin-colour columns of one source, the pseudoscalar and
  midpoint correlators and their ratio (the paper's m_res(t), with the
  midpoint density of the Shamir definition):
      C_PP(t) = sum_{x in t} sum_cols |q|^2,   C_mp(t) = sum_{x in t} sum_cols |Q|^2,
      m_res(t) = C_mp(t) / C_PP(t).
  Both are products of a propagator with its gamma5-adjoint, so they are
  sums of squared moduli.  The same sum over any 4D fields (a propagator's
  columns with the sink smeared, say) is the pseudoscalar correlator of
  those fields.

Chiral basis, g5 = diag(1, 1, -1, -1): P+ keeps spins 0, 1 and P- spins 2, 3.
Layouts: links U[t, z, y, x, mu, a, b], 4D spinors [t, z, y, x, spin, colour],
5D spinors [s, t, z, y, x, spin, colour], complex128.
"""
import numpy as np

from oracle import Action, dw4

# array axis of the direction mu in a field indexed [t, z, y, x, ...]
_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}
_PP = np.array([1.0, 1.0, 0.0, 0.0])[:, None]     # P+ on [spin, colour]
_PM = np.array([0.0, 0.0, 1.0, 1.0])[:, None]     # P-


def laplacian(U, psi):
    """Covariant spatial Laplacian of a 4D spinor field (periodic in x, y, z)."""
    out = -6.0 * psi
    for mu in range(3):
        Umu = U[..., mu, :, :]
        fwd = np.roll(psi, -1, axis=_AXIS[mu])                       # psi(x + mu)
        out = out + np.einsum("tzyxab,tzyxsb->tzyxsa", Umu, fwd)
        bwd_link = np.roll(Umu, 1, axis=_AXIS[mu])                    # U_mu(x - mu)
        bwd = np.roll(psi, 1, axis=_AXIS[mu])                         # psi(x - mu)
        out = out + np.einsum("tzyxba,tzyxsb->tzyxsa", np.conj(bwd_link), bwd)
    return out


def gauss_smear(U, psi, sigma, niter):
    """(1 + sigma^2/(4 niter) Delta)^niter psi, niter explicit steps."""
    out = np.array(psi, dtype=np.complex128, copy=True)
    if niter <= 0:
        return out
    kappa = sigma * sigma / (4.0 * niter)
    for _ in range(int(niter)):
        out = out + kappa * laplacian(U, out)
    return out


def wall_source(act: Action, U, eta):
    """b = (1 - c5 D_W) Pbar eta: a 5D right-hand side from a 4D source."""
    L5 = act.L5
    b = np.zeros((L5,) + eta.shape, dtype=np.complex128)
    for s, proj in ((L5 - 1, _PM), (0, _PP)):
        e = proj * eta
        b[s] += e - act.c5 * dw4(act, U, e)
    return b


def project_wall(x5):
    """q = P- x_0 + P+ x_{L5-1}: the 4D quark field at the domain walls."""
    return _PM * x5[0] + _PP * x5[-1]


def project_mid(x5):
    """Q = P- x_{L5/2} + P+ x_{L5/2-1}: the 4D field at the midpoint of L5."""
    L5 = x5.shape[0]
    if L5 % 2:
        raise ValueError("the midpoint needs an even L5")
    return _PM * x5[L5 // 2] + _PP * x5[L5 // 2 - 1]


def correlators(x5_cols):
    """(C_PP, C_mp, m_res) per time slice from the 5D solutions of the
    columns of one source (any number of columns, all summed)."""
    cpp = 0.0
    cmp_ = 0.0
    for x5 in x5_cols:
        q, Q = project_wall(x5), project_mid(x5)
        cpp = cpp + np.sum(np.abs(q) ** 2, axis=(1, 2, 3, 4, 5))
        cmp_ = cmp_ + np.sum(np.abs(Q) ** 2, axis=(1, 2, 3, 4, 5))
    return cpp, cmp_, cmp_ / cpp


def pion_correlator(fields4d):
    """sum over each time slice's sites, spins and colours, and over the
    given 4D fields (the columns of one source, at the sink as they are or
    smeared), of |q|^2: the pseudoscalar correlator of those columns."""
    c = 0.0
    for q in fields4d:
        c = c + np.sum(np.abs(q) ** 2, axis=(1, 2, 3, 4, 5))
    return c


def point_source(dims, site, spin, colour):
    """Unit 4D source at site (t, z, y, x) in one spin and colour."""
    T, Z, Y, X = dims[3], dims[2], dims[1], dims[0]
    eta = np.zeros((T, Z, Y, X, 4, 3), dtype=np.complex128)
    eta[tuple(site) + (spin, colour)] = 1.0
    return eta
