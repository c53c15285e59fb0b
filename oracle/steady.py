"""Direct solve of the steady discrete flow problem (test infrastructure only).

At steady state the ACM iteration of Sec. 2.3 balances momentum with the
RBF-FD operators of Sec. 2.1,

    nu (Lap v)_i - ((v.grad) v)_i - (grad p)_i / rho + g = 0     interior i,
    (div v)_i = kappa                                             interior i,
    (dn p)_b = 0                                                  boundary b,
    v_b = 0,   mean(p) = 0,

where kappa is one uniform constant: the discrete divergence is not exactly
conservative, and a uniform residual only makes the pressure gauge drift,
which no gradient sees.  This module assembles that sparse system from the
oracle's weights and solves it directly (Picard iterations for the advection
term; with advection=False it is the Stokes problem).  It is an algorithm
independent of time stepping, used to pin the oracle's steady permeability and
drag against the dilute-array closed form.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def steady_solve(n_int, sten, w, sten_n, wn, nu=1.0, rho=1.0, g=(1.0, 0.0, 0.0), advection=False, picard=8,
                 tol=1e-12):
    """w: [N][4][nl] (dx, dy, dz, lap) for every node; sten_n/wn: Neumann rows
    of the boundary nodes.  Returns v [N][3], p [N], kappa."""
    sten = np.asarray(sten)
    N, nl = sten.shape
    ni = int(n_int)
    nb = N - ni
    nv = 3 * ni
    ncol = nv + N + 1
    g = np.asarray(g, dtype=np.float64)

    rows_i = np.repeat(np.arange(ni), nl)
    cols_s = sten[:ni].ravel()
    interior_nb = cols_s < ni

    def base_blocks():
        blocks = []
        # pressure gradient in momentum rows, continuity rows
        for a in range(3):
            wa = w[:ni, a, :].ravel()
            blocks.append((a * ni + rows_i, nv + cols_s, -wa / rho))
            m = interior_nb
            blocks.append((nv + rows_i[m], a * ni + cols_s[m], wa[m]))
        blocks.append((nv + np.arange(ni), np.full(ni, ncol - 1), -np.ones(ni)))
        # Neumann rows of boundary nodes
        if nb:
            rb = np.repeat(np.arange(nb), nl)
            blocks.append((nv + ni + rb, nv + np.asarray(sten_n).ravel(), np.asarray(wn).ravel()))
        # gauge row
        blocks.append((np.full(N, nv + N), nv + np.arange(N), np.full(N, 1.0 / N)))
        return blocks

    fixed = base_blocks()
    v = np.zeros((N, 3))
    rhs = np.zeros(ncol)
    for a in range(3):
        rhs[a * ni:(a + 1) * ni] = -g[a]
    x = None
    for it in range(picard if advection else 1):
        blocks = list(fixed)
        for a in range(3):
            m = interior_nb
            coef = nu * w[:ni, 3, :].ravel()
            if advection:
                # (v*.grad) v_a with v* frozen: sum_c v*_c,i (d_c v_a)_i
                for c in range(3):
                    coef = coef - np.repeat(v[:ni, c], nl) * w[:ni, c, :].ravel()
            blocks.append((a * ni + rows_i[m], a * ni + cols_s[m], coef[m]))
        r = np.concatenate([b[0] for b in blocks])
        c = np.concatenate([b[1] for b in blocks])
        d = np.concatenate([b[2] for b in blocks])
        A = sp.csc_matrix((d, (r, c)), shape=(ncol, ncol))
        x_new = spla.splu(A, permc_spec="COLAMD").solve(rhs)
        v_new = np.zeros((N, 3))
        for a in range(3):
            v_new[:ni, a] = x_new[a * ni:(a + 1) * ni]
        done = x is not None and np.abs(v_new - v).max() <= tol * max(np.abs(v_new).max(), 1e-300)
        v, x = v_new, x_new
        if done:
            break
    p = x[nv:nv + N].copy()
    return v, p, float(x[-1])
