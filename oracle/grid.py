"""Uniform MAC grid and its difference operators (oracle, test infrastructure).

Cell-centred scalars q (phi, mu, p, rho, eta) and face-normal vectors F_a
(velocity, fluxes).  Face entry c of axis a sits between cells c - e_a and c.
On a walled axis the face with index 0 along that axis is the wall; the other
wall face (index n_a) is not stored and is zero by definition.

Definitions (all written out, no shared helpers with the GPU library):
  G_a q   = (q_c - q_{c-e_a}) / h              gradient, zero on wall faces
                                               (no-flux / Neumann, boundary
                                               conditions of the mass-
                                               conservation proposition)
  D F     = sum_a (F_{c+e_a} - F_c) / h        divergence, wall faces carry
                                               zero flux
  A_a q   = (q_c + q_{c-e_a}) / 2              cell-to-face average
  L       = D o G                              Laplacian
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np


class MACGrid:
    def __init__(self, n: Sequence[int], h: float, periodic: Sequence[bool]):
        self.n = tuple(int(x) for x in n)
        self.dim = len(self.n)
        self.shape = tuple(reversed(self.n))
        self.h = float(h)
        self.periodic = tuple(bool(x) for x in periodic)
        assert len(self.periodic) == self.dim

    # numpy axis of grid axis a (x is the last / fastest numpy axis)
    def ax(self, a: int) -> int:
        return self.dim - 1 - a

    def index(self, a: int) -> np.ndarray:
        """Integer index along grid axis a, broadcast to the cell shape."""
        sh = [1] * self.dim
        sh[self.ax(a)] = self.n[a]
        return np.broadcast_to(np.arange(self.n[a]).reshape(sh), self.shape)

    def shift(self, q: np.ndarray, a: int, s: int, fill: float = 0.0) -> np.ndarray:
        """Return r with r[c] = q[c + s e_a]; outside a walled axis r = fill."""
        if self.periodic[a]:
            return np.roll(q, -s, axis=self.ax(a))
        r = np.full_like(q, fill)
        n = self.n[a]
        src = [slice(None)] * self.dim
        dst = [slice(None)] * self.dim
        if s >= 0:
            src[self.ax(a)] = slice(s, n)
            dst[self.ax(a)] = slice(0, n - s)
        else:
            src[self.ax(a)] = slice(0, n + s)
            dst[self.ax(a)] = slice(-s, n)
        r[tuple(dst)] = q[tuple(src)]
        return r

    def wall_face_mask(self, a: int) -> np.ndarray:
        """True on the stored wall faces of axis a (index 0 of a walled axis)."""
        if self.periodic[a]:
            return np.zeros(self.shape, dtype=bool)
        return self.index(a) == 0

    def grad(self, q: np.ndarray, a: int) -> np.ndarray:
        g = (q - self.shift(q, a, -1)) / self.h
        g[self.wall_face_mask(a)] = 0.0
        return g

    def div(self, F: List[np.ndarray]) -> np.ndarray:
        out = np.zeros(self.shape)
        for a in range(self.dim):
            Fm = np.where(self.wall_face_mask(a), 0.0, F[a])
            Fp = self.shift(Fm, a, +1, fill=0.0)  # upper wall face: zero flux
            out += (Fp - Fm) / self.h
        return out

    def avg(self, q: np.ndarray, a: int) -> np.ndarray:
        """Face average; on a stored wall face the adjacent cell value."""
        qm = self.shift(q, a, -1)
        w = self.wall_face_mask(a)
        qm = np.where(w, q, qm)
        return 0.5 * (q + qm)

    def lap(self, q: np.ndarray) -> np.ndarray:
        return self.div([self.grad(q, a) for a in range(self.dim)])

    def coords(self) -> List[np.ndarray]:
        return [(self.index(a) + 0.5) * self.h for a in range(self.dim)]

    # ---- sparse matrices of the same operators (for identities / direct solves)
    def cell_index(self) -> np.ndarray:
        return np.arange(int(np.prod(self.shape))).reshape(self.shape)

    def grad_matrix(self, a: int):
        """Sparse G_a: cells -> faces of axis a (rows of wall faces are empty)."""
        import scipy.sparse as sp
        N = int(np.prod(self.shape))
        idx = self.cell_index()
        im = self.shift(idx, a, -1, fill=-1)
        ok = ~self.wall_face_mask(a)
        rows = idx[ok]
        cols_p = idx[ok]
        cols_m = im[ok]
        data = np.concatenate([np.full(rows.size, 1.0 / self.h), np.full(rows.size, -1.0 / self.h)])
        return sp.csr_matrix((data, (np.concatenate([rows, rows]), np.concatenate([cols_p, cols_m]))),
                             shape=(N, N))

    def div_matrix(self, a: int):
        """Sparse D restricted to axis a: faces of axis a -> cells."""
        import scipy.sparse as sp
        N = int(np.prod(self.shape))
        idx = self.cell_index()
        ip = self.shift(idx, a, +1, fill=-1)
        wall = self.wall_face_mask(a)
        rows, cols, data = [], [], []
        # + F_{c+e_a}/h  (skip the unstored upper wall face)
        ok = ip >= 0
        rows.append(idx[ok]); cols.append(ip[ok]); data.append(np.full(ok.sum(), 1.0 / self.h))
        # - F_c/h  (skip stored wall faces)
        ok = ~wall
        rows.append(idx[ok]); cols.append(idx[ok]); data.append(np.full(ok.sum(), -1.0 / self.h))
        return sp.csr_matrix((np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(N, N))

    def lap_matrix(self):
        L = None
        for a in range(self.dim):
            t = self.div_matrix(a) @ self.grad_matrix(a)
            L = t if L is None else L + t
        return L.tocsr()
