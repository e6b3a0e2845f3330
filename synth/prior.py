"""Seeded stand-in for the learned Fields-of-Experts prior.

The trained filters and weights of the paper (Fig. "filters", Section 3.2)
are not published.  The paper builds its filters from a modified DCT basis
with the constant atom removed, so that every filter is zero-mean
(eq. 2.11 and Section 2.6).  The stand-in keeps that structure: with
B the (m^2 - 1) x m^2 matrix of non-constant orthonormal 2-D DCT-II atoms
and Q the orthogonal factor of a seeded Gaussian matrix (QR with the sign of
R's diagonal folded into Q), the filters are the rows of Q[:N_f] @ B.  They
are orthonormal, zero-mean, unit-norm and in general not symmetric under a
180-degree rotation, which keeps a convolution/correlation mix-up visible.
Weights alpha_i are log-uniform on [0.1, 10].

Filters are returned as float32 correlation taps k[i][a][b]; the float32
values are the inputs both sides receive.
"""
import numpy as np


def dct_basis_no_dc(m):
    """(m*m - 1, m, m) orthonormal 2-D DCT-II atoms without the constant one."""
    n = np.arange(m)
    c = np.cos(np.pi * (2 * n[None, :] + 1) * n[:, None] / (2.0 * m))
    c *= np.sqrt(2.0 / m)
    c[0] /= np.sqrt(2.0)
    atoms = [np.outer(c[i], c[j]) for i in range(m) for j in range(m)
             if not (i == 0 and j == 0)]
    return np.stack(atoms)


def make_prior(seed, m, n_filters, scale=1.0, atoms_only=False):
    """Return (filters float32 [N_f, m, m], weights float32 [N_f])."""
    g = np.random.Generator(np.random.PCG64(seed))
    basis = dct_basis_no_dc(m).reshape(m * m - 1, m * m)
    nb = basis.shape[0]
    if n_filters > nb:
        raise ValueError("at most m*m-1 zero-mean filters")
    if atoms_only:
        q = np.eye(nb)
    else:
        q, rr = np.linalg.qr(g.standard_normal((nb, nb)))
        q = q * np.sign(np.diag(rr))[None, :]
    k = (q[:n_filters] @ basis).reshape(n_filters, m, m) * scale
    w = 10.0 ** g.uniform(-1.0, 1.0, n_filters)
    return k.astype(np.float32), w.astype(np.float32)
