"""Wilson gradient flow of SU(3) gauge links -- FP64 CPU reference.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU baseline of
the benchmark use this module; the library never does.  It shares no code
with the HIP path.

The paper smooths its gauge ensembles by the gradient flow before the
valence solves, at flow time t_gf = 1 in lattice units (Sec. III, "Gradient-
flow smearing"), citing Luscher's Wilson flow.  That flow is

    dV_t(x, mu)/dt = Z(V_t)(x, mu) V_t(x, mu),
    Z = -g0^2 d_{x,mu} S_w,   S_w = (1/g0^2) sum over oriented plaquettes p of Re tr(1 - V(p)),

whose right-hand side works out to the traceless antihermitian projection

    Z_mu(x) = -1/2 (Omega - Omega^+) + 1/6 tr(Omega - Omega^+),
    Omega_mu(x) = U_mu(x) sum_{nu != mu} [ U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
                                          + U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu) ],

integrated with the third-order Runge-Kutta scheme of the same reference:

    W0 = V_t,  Z_i = eps Z(W_i),
    W1 = exp(1/4 Z0) W0,
    W2 = exp(8/9 Z1 - 17/36 Z0) W1,
    V_{t+eps} = exp(3/4 Z2 - 8/9 Z1 + 17/36 Z0) W2.

Layout: U[t, z, y, x, mu, a, b] complex128, mu = 0..3 for x, y, z, t; all
directions periodic (the gauge field is).  The exponential of a traceless
antihermitian matrix X is taken from the eigen-decomposition of the
Hermitian -iX.
"""
import numpy as np

# array axis of the direction mu in U[t, z, y, x, ...]
_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def _shift(f, mu, k):
    """f(x + k mu) for a field indexed [t, z, y, x, ...]."""
    return np.roll(f, -k, axis=_AXIS[mu])


def _dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def omega(U):
    """Omega_mu(x) for every link: the link times the sum of its six staples."""
    out = np.empty_like(U)
    for mu in range(4):
        S = np.zeros(U.shape[:4] + (3, 3), dtype=np.complex128)
        for nu in range(4):
            if nu == mu:
                continue
            Unu, Umu = U[..., nu, :, :], U[..., mu, :, :]
            up = _shift(Unu, mu, 1) @ _dag(_shift(Umu, nu, 1)) @ _dag(Unu)
            Unu_m = _shift(Unu, nu, -1)
            down = _dag(_shift(Unu_m, mu, 1)) @ _dag(_shift(Umu, nu, -1)) @ Unu_m
            S = S + up + down
        out[..., mu, :, :] = U[..., mu, :, :] @ S
    return out


def force(U):
    """Z(U) = -g0^2 d S_w: the traceless antihermitian matrix of every link."""
    Om = omega(U)
    A = Om - _dag(Om)
    tr = np.trace(A, axis1=-2, axis2=-1)
    return -0.5 * A + (tr / 6.0)[..., None, None] * np.eye(3)


def expm_ah(X):
    """exp(X) for traceless antihermitian 3x3 matrices X (any leading shape)."""
    w, v = np.linalg.eigh(-1j * X)          # -iX is Hermitian: X = i v diag(w) v^+
    return (v * np.exp(1j * w)[..., None, :]) @ _dag(v)


def wilson_action(U):
    """g0^2 S_w = sum over oriented plaquettes of Re tr(1 - U(p)), i.e. twice
    the sum over the unoriented ones."""
    s = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Umu, Unu = U[..., mu, :, :], U[..., nu, :, :]
            P = Umu @ _shift(Unu, mu, 1) @ _dag(_shift(Umu, nu, 1)) @ _dag(Unu)
            s += 2.0 * np.sum(3.0 - np.trace(P, axis1=-2, axis2=-1).real)
    return float(s)


def plaquette(U):
    """Average plaquette (1/3) Re tr U(p) over sites and the six planes."""
    V = int(np.prod(U.shape[:4]))
    return 1.0 - wilson_action(U) / (2.0 * 6.0 * 3.0 * V)


def flow_step(U, eps):
    """One Runge-Kutta step of flow time eps."""
    Z0 = eps * force(U)
    W1 = expm_ah(0.25 * Z0) @ U
    Z1 = eps * force(W1)
    W2 = expm_ah(8.0 / 9.0 * Z1 - 17.0 / 36.0 * Z0) @ W1
    Z2 = eps * force(W2)
    return expm_ah(0.75 * Z2 - 8.0 / 9.0 * Z1 + 17.0 / 36.0 * Z0) @ W2


def flow(U, eps, nsteps):
    """nsteps Runge-Kutta steps of size eps (flow time nsteps * eps)."""
    V = np.array(U, dtype=np.complex128, copy=True)
    for _ in range(int(nsteps)):
        V = flow_step(V, eps)
    return V
