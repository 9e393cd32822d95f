"""Independent sparse-matrix assembly of the Moebius operator, for pinning the oracle.

This builds D_W and D5 as explicit sparse matrices from Kronecker products of
shift matrices, link blocks, gamma matrices and fifth-dimension shift
matrices.  It is written from the operator definitions (paper Sec. II: the
Wilson operator at height M5 and the Moebius kernel; the domain-wall fifth
dimension of Sec. I), shares no code with the oracle's stencil loops, and is
only used by the tests.

Index order matches the host canonical layout: (s, t, z, y, x, spin, colour),
flattened C-order, so that a matrix here acts on ``psi.ravel()``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Chiral-basis Euclidean gamma matrices, typed from their definition:
# g_k = [[0, -i s_k], [i s_k, 0]] (k = 1, 2, 3), g_4 = [[0, 1], [1, 0]].
SIGMA = [np.array([[0, 1], [1, 0]], complex),
         np.array([[0, -1j], [1j, 0]], complex),
         np.array([[1, 0], [0, -1]], complex)]


def gammas():
    z = np.zeros((2, 2), complex)
    g = [np.block([[z, -1j * s], [1j * s, z]]) for s in SIGMA]
    g.append(np.block([[z, np.eye(2)], [np.eye(2), z]]))
    return g


G5 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(complex)
PPLUS = (np.eye(4) + G5) / 2
PMINUS = (np.eye(4) - G5) / 2


def _site_index(dims):
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel(), t.ravel()


def link_hop_blocks(U, dims, antiperiodic_t=True):
    """Per direction, sparse (3V x 3V) forward and backward colour hops.

    F_mu[(x,a),(x+mu,b)] = bc * U_mu(x)_{ab}
    K_mu[(x,a),(x-mu,b)] = bc * conj(U_mu(x-mu)_{ba})
    """
    X, Y, Z, T = dims
    L = [X, Y, Z, T]
    V = X * Y * Z * T
    xs = list(_site_index(dims))
    lex = xs[0] + X * (xs[1] + Y * (xs[2] + Z * xs[3]))
    Uf = U.reshape(V, 4, 3, 3)
    out = []
    for mu in range(4):
        c = [a.copy() for a in xs]
        c[mu] = (xs[mu] + 1) % L[mu]
        fwd = c[0] + X * (c[1] + Y * (c[2] + Z * c[3]))
        bc_f = np.where((xs[mu] == L[mu] - 1) & (mu == 3) & antiperiodic_t, -1.0, 1.0)
        c = [a.copy() for a in xs]
        c[mu] = (xs[mu] - 1) % L[mu]
        bwd = c[0] + X * (c[1] + Y * (c[2] + Z * c[3]))
        bc_b = np.where((xs[mu] == 0) & (mu == 3) & antiperiodic_t, -1.0, 1.0)
        rows, cols, vf = [], [], []
        rb, cb, vb = [], [], []
        for a in range(3):
            for b in range(3):
                rows.append(3 * lex + a)
                cols.append(3 * fwd + b)
                vf.append(bc_f * Uf[lex, mu, a, b])
                rb.append(3 * lex + a)
                cb.append(3 * bwd + b)
                vb.append(bc_b * np.conj(Uf[bwd, mu, b, a]))
        F = sp.csr_matrix((np.concatenate(vf), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(3 * V, 3 * V))
        K = sp.csr_matrix((np.concatenate(vb), (np.concatenate(rb), np.concatenate(cb))),
                          shape=(3 * V, 3 * V))
        out.append((F, K))
    return out


def _spin_between(M_sitecol, S_spin, V):
    """Operator acting as M on (site, colour) and S on spin, in (site, spin, colour) order."""
    # reorder: (site, colour) x (spin) -> (site, spin, colour)
    M = sp.csr_matrix(M_sitecol)
    big = sp.kron(M, sp.csr_matrix(S_spin), format="csr")  # index (site,colour,spin)
    perm = np.arange(12 * V).reshape(V, 3, 4).transpose(0, 2, 1).ravel()
    # perm[k] = (site,colour,spin)-index of the k-th (site,spin,colour) entry
    return big[perm][:, perm]


def dslash_matrix(U, dims, antiperiodic_t=True, dag=False):
    V = int(np.prod(dims))
    g = gammas()
    sg = -1.0 if dag else 1.0
    D = sp.csr_matrix((12 * V, 12 * V), dtype=complex)
    for mu, (F, K) in enumerate(link_hop_blocks(U, dims, antiperiodic_t)):
        D = D + _spin_between(F, np.eye(4) - sg * g[mu], V) + _spin_between(K, np.eye(4) + sg * g[mu], V)
    return D.tocsr()


def dw_matrix(U, dims, M5, antiperiodic_t=True):
    V = int(np.prod(dims))
    return (sp.identity(12 * V, dtype=complex) * (4.0 - M5)
            - 0.5 * dslash_matrix(U, dims, antiperiodic_t)).tocsr()


def c5_matrix(L5, mq):
    """Fifth-dimension shifts (L5 x L5) for the two chiralities.

    Positive chirality reads slice s-1, negative chirality reads s+1; the
    wrap-around entries carry -m_q.
    """
    Sp = np.zeros((L5, L5))
    Sm = np.zeros((L5, L5))
    for s in range(L5):
        if s >= 1:
            Sp[s, s - 1] = 1.0
        else:
            Sp[s, L5 - 1] = -mq
        if s + 1 < L5:
            Sm[s, s + 1] = 1.0
        else:
            Sm[s, 0] = -mq
    return Sp, Sm


def C_matrix(dims, L5, mq):
    V = int(np.prod(dims))
    Sp, Sm = c5_matrix(L5, mq)
    site = sp.identity(V, format="csr")
    col = sp.identity(3, format="csr")
    return (sp.kron(sp.kron(sp.kron(Sp, site), sp.csr_matrix(PPLUS)), col)
            + sp.kron(sp.kron(sp.kron(Sm, site), sp.csr_matrix(PMINUS)), col)).tocsr()


def d5_matrix(U, dims, L5, M5, b5, c5, mq, antiperiodic_t=True):
    """D5 = (1_s x D_W)(b5 + c5 C) + 1 - C."""
    V = int(np.prod(dims))
    n = 12 * V * L5
    DW = dw_matrix(U, dims, M5, antiperiodic_t)
    DW5 = sp.kron(sp.identity(L5), DW, format="csr")
    Cm = C_matrix(dims, L5, mq)
    Id = sp.identity(n, dtype=complex, format="csr")
    return (DW5 @ (b5 * Id + c5 * Cm) + Id - Cm).tocsr()


def gamma5_field(n_sites):
    return sp.kron(sp.kron(sp.identity(n_sites), sp.csr_matrix(G5)), sp.identity(3), format="csr")


def parity_vector(dims):
    """4D parity of each canonical site index."""
    x, y, z, t = _site_index(dims)
    return (x + y + z + t) % 2
