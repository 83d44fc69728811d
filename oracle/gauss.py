"""FP64 oracle of the Gauss'-law weight correction (Sec. 2.4.1), test
infrastructure only (like the rest of this package; shares nothing with the
library).

Mesh: periodic, nx cells in 1D (dx = 1) or nx * ny cells in 2D (dx = 2, cell
c at (c % nx, c // nx)), unit cell size in index units; cell i has centre
X_i = i + 1/2.  A particle of cell c with cell-local position x in [0, 1)^dx
sits at X = (cell coordinates) + x.

  deposit      D_i = sum_p w_p S2(X_i - X_p): the charge a particle set puts
               on mesh cell i with the second-order (quadratic) B-spline
               S2, a partition of unity; the paper's rho_i times the cell
               volume, with unit charge q.
  mass matrix  M_ij = sum_{p in cell j} S2(X_i - X_p): S0 (top hat) picks the
               particles of cell j, eq. p-weight-correction.
  correction   M dA = D_target - D(w), then w'_p = w_p + dA_{cell(p)} (eq.
               new-p-weight), so that D(w') = D_target.

The linear system is solved with a sparse direct solver (a library step).
"""
from __future__ import annotations

import numpy as np


def s2(s):
    """Quadratic B-spline: 3/4 - s^2 for |s| <= 1/2, (3/2 - |s|)^2 / 2 for
    1/2 <= |s| <= 3/2, 0 beyond."""
    a = np.abs(np.asarray(s, dtype=np.float64))
    return np.where(a <= 0.5, 0.75 - a * a, np.where(a <= 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def _mesh(n_cells, dx, nx):
    ny = n_cells // nx if dx == 2 else 1
    if dx == 2 and nx * ny != n_cells:
        raise ValueError("nx must divide n_cells on a 2D mesh")
    if dx not in (1, 2):
        raise ValueError("dx must be 1 or 2")
    return nx if dx == 2 else n_cells, ny


def _cell_of(cell_off):
    return np.repeat(np.arange(len(cell_off) - 1), np.diff(cell_off))


def _stencil(x, cell_off, dx, nx):
    """For every particle: the mesh cells of its S2 stencil (3 in 1D, 9 in
    2D, periodic) and the weights S2(X_i - X_p)."""
    n_cells = len(cell_off) - 1
    nx, ny = _mesh(n_cells, dx, nx)
    c = _cell_of(cell_off)
    x = np.asarray(x, dtype=np.float64).reshape(len(c), dx)
    if dx == 1:
        cx = c
        idx, wt = [], []
        for o in (-1, 0, 1):
            s = (cx + o + 0.5) - (cx + x[:, 0])
            idx.append((cx + o) % nx)
            wt.append(s2(s))
        return np.stack(idx, 1), np.stack(wt, 1)
    cx, cy = c % nx, c // nx
    idx, wt = [], []
    for oy in (-1, 0, 1):
        for ox in (-1, 0, 1):
            sx = (cx + ox + 0.5) - (cx + x[:, 0])
            sy = (cy + oy + 0.5) - (cy + x[:, 1])
            idx.append(((cy + oy) % ny) * nx + (cx + ox) % nx)
            wt.append(s2(sx) * s2(sy))
    return np.stack(idx, 1), np.stack(wt, 1)


def deposit(x, w, cell_off, dx, nx):
    """D_i = sum_p w_p S2(X_i - X_p) on the periodic mesh (one value per cell)."""
    n_cells = len(cell_off) - 1
    idx, wt = _stencil(x, cell_off, dx, nx)
    out = np.zeros(n_cells)
    np.add.at(out, idx.ravel(), (np.asarray(w, dtype=np.float64)[:, None] * wt).ravel())
    return out


def mass_matrix(x, cell_off, dx, nx):
    """M_ij = sum_{p in cell j} S2(X_i - X_p) as a scipy sparse matrix."""
    import scipy.sparse as sp
    n_cells = len(cell_off) - 1
    idx, wt = _stencil(x, cell_off, dx, nx)
    cols = np.repeat(_cell_of(cell_off), idx.shape[1])
    return sp.csr_matrix((wt.ravel(), (idx.ravel(), cols)), shape=(n_cells, n_cells))


def gauss_correct(x, w, cell_off, d_target, dx, nx):
    """Per-cell weight corrections dA and corrected weights w' with
    deposit(w') = d_target (every cell must hold a particle)."""
    import scipy.sparse.linalg as spl
    if (np.diff(cell_off) <= 0).any():
        raise ValueError("every cell needs at least one particle")
    M = mass_matrix(x, cell_off, dx, nx).tocsc()
    b = np.asarray(d_target, dtype=np.float64) - deposit(x, w, cell_off, dx, nx)
    dA = spl.spsolve(M, b)
    return dA, np.asarray(w, dtype=np.float64) + dA[_cell_of(cell_off)]
