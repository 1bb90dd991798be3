"""Sizes, mode sets and grids of the discretised cavity problem (oracle; test only).

Paper: Section 3 (Fourier expansions (E123F), mode sets N1, N2, N3 after (ode3x3),
uniform z-grid before (dfE1M)), Section 4 (layers, interfaces on grid nodes), Section 5
(truncation radius R = sqrt(2) * max side, FFT convolution on a periodic box).

Readings (where the paper leaves a choice open):
* M = Nx - 1 and N = Ny - 1 Fourier modes; the z-grid has Nz intervals, h = c / Nz, the
  aperture is node Nz (the paper's J+1) and the bottom node 0.
* Layers are listed bottom to top and interfaces sit on nodes.  By default every layer
  has the common step h = c / Nz (the paper's two-layer derivation assumes one h).  With
  layer thicknesses d_l given, layer l has its own step h_l = d_l / Nz_l (Example 3's
  table assigns different interval counts to layers of different thickness); the
  interface rows then weight the one-sided differences by their own steps (see
  ``columns``), and h denotes the top layer's step, the one the aperture rows use.
* TBC quadrature grid: s*Nx x s*Ny intervals on the aperture (s >= 1), trapezoid weights.
* FFT box per axis: P = smallest 5-smooth integer >= ceil((side + R) / hq), L = P * hq,
  which keeps the kernel truncated at R from wrapping onto the aperture.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


def next_5smooth(n: int) -> int:
    """Smallest integer >= n whose only prime factors are 2, 3 and 5."""
    n = max(int(n), 1)
    while True:
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            return n
        n += 1


@dataclass
class Problem:
    a: float
    b: float
    c: float
    nx: int
    ny: int
    nz: int
    layer_nz: Tuple[int, ...]
    layer_eps: Tuple[complex, ...]
    k: float
    s: int = 1
    layer_depth: Optional[Tuple[float, ...]] = None
    # derived
    M: int = field(init=False)
    N: int = field(init=False)
    h: float = field(init=False)
    layer_h: Tuple[float, ...] = field(init=False)

    def __post_init__(self):
        if self.nx < 2 or self.ny < 2 or self.nz < 1:
            raise ValueError("need nx, ny >= 2 and nz >= 1")
        if sum(self.layer_nz) != self.nz or min(self.layer_nz) < 1:
            raise ValueError("layer_nz must be positive and sum to nz")
        self.layer_nz = tuple(int(v) for v in self.layer_nz)
        self.layer_eps = tuple(complex(v) for v in self.layer_eps)
        self.M = self.nx - 1
        self.N = self.ny - 1
        if self.layer_depth is None:
            self.layer_h = tuple(self.c / self.nz for _ in self.layer_nz)
        else:
            d = tuple(float(v) for v in self.layer_depth)
            if len(d) != len(self.layer_nz) or min(d) <= 0.0:
                raise ValueError("layer_depth needs one positive thickness per layer")
            if abs(sum(d) - self.c) > 1e-12 * self.c:
                raise ValueError("layer thicknesses must sum to c")
            self.layer_depth = d
            self.layer_h = tuple(dl / nl for dl, nl in zip(d, self.layer_nz))
        self.h = self.layer_h[-1]

    @classmethod
    def from_cavity(cls, cav) -> "Problem":
        depth = getattr(cav, "layer_depth", None)
        return cls(cav.a, cav.b, cav.c, cav.nx, cav.ny, cav.nz, tuple(cav.layer_nz),
                   tuple(cav.layer_eps), cav.k, cav.tbc_oversample,
                   None if depth is None else tuple(depth))

    # -- Fourier modes (Section 3, (E123F)) -------------------------------------------
    @property
    def mu(self) -> np.ndarray:
        """mu_m = m pi / a, m = 0..M."""
        return np.pi * np.arange(self.M + 1) / self.a

    @property
    def nu(self) -> np.ndarray:
        """nu_n = n pi / b, n = 0..N."""
        return np.pi * np.arange(self.N + 1) / self.b

    def masks(self):
        """Boolean (M+1) x (N+1) masks of the mode sets N1 (E1), N2 (E2), N3 (E3)."""
        m = np.arange(self.M + 1)[:, None]
        n = np.arange(self.N + 1)[None, :]
        n1 = np.broadcast_to(n >= 1, (self.M + 1, self.N + 1)).copy()
        n2 = np.broadcast_to(m >= 1, (self.M + 1, self.N + 1)).copy()
        n3 = (m >= 1) & (n >= 1)
        return n1, n2, n3

    @property
    def n_ap(self) -> int:
        """Aperture unknowns (M+1)N + M(N+1) + MN."""
        M, N = self.M, self.N
        return (M + 1) * N + M * (N + 1) + M * N

    @property
    def unknowns(self) -> int:
        """Unknowns per right-hand side: aperture modes times z-levels 1..Nz."""
        return self.n_ap * self.nz

    # -- aperture vector: paper ordering (Appendix A): E1, E2, E3, each m-major ----------
    def pack(self, e1, e2, e3) -> np.ndarray:
        n1, n2, n3 = self.masks()
        return np.concatenate([e1[n1], e2[n2], e3[n3]])

    def unpack(self, x):
        n1, n2, n3 = self.masks()
        shape = (self.M + 1, self.N + 1)
        out = []
        off = 0
        for msk in (n1, n2, n3):
            arr = np.zeros(shape, dtype=complex)
            cnt = int(msk.sum())
            arr[msk] = x[off:off + cnt]
            off += cnt
            out.append(arr)
        return tuple(out)

    # -- layers on the z-grid (Section 4) ------------------------------------------------
    @property
    def interfaces(self) -> List[int]:
        """Interface node indices, bottom to top (nodes between consecutive layers)."""
        return [int(v) for v in np.cumsum(self.layer_nz)[:-1]]

    def node_kind(self):
        """For nodes j = 0..Nz: ('interior', layer) or ('interface', lower, upper) or
        ('bottom',) / ('aperture',)."""
        kinds = [None] * (self.nz + 1)
        kinds[0] = ("bottom",)
        kinds[self.nz] = ("aperture",)
        start = 0
        for ell, nzl in enumerate(self.layer_nz):
            for j in range(start + 1, start + nzl):
                kinds[j] = ("interior", ell)
            start += nzl
            if ell < len(self.layer_nz) - 1:
                kinds[start] = ("interface", ell, ell + 1)
        return kinds

    def h_layer(self, ell: int) -> float:
        """Grid step of layer ell."""
        return self.layer_h[ell]

    def z_nodes(self) -> np.ndarray:
        """Heights of the nodes j = 0..Nz above the bottom."""
        steps = np.concatenate([np.full(nl, hl) for nl, hl in zip(self.layer_nz, self.layer_h)])
        return np.concatenate([[0.0], np.cumsum(steps)])

    def kappa2(self, ell: int) -> complex:
        """kappa^2 = k^2 eps_r in layer ell (non-magnetic medium)."""
        return self.k ** 2 * self.layer_eps[ell]

    def lam(self, ell: int) -> np.ndarray:
        """kappa_ell^2 - mu_m^2 - nu_n^2 on the (M+1) x (N+1) mode grid."""
        return self.kappa2(ell) - self.mu[:, None] ** 2 - self.nu[None, :] ** 2

    # -- TBC quadrature grid and FFT box (Section 5) -------------------------------------
    @property
    def nq(self) -> Tuple[int, int]:
        return self.s * self.nx, self.s * self.ny

    @property
    def hq(self) -> Tuple[float, float]:
        return self.a / (self.s * self.nx), self.b / (self.s * self.ny)

    @property
    def R(self) -> float:
        return math.sqrt(2.0) * max(self.a, self.b)

    @property
    def box(self) -> Tuple[int, int]:
        hq1, hq2 = self.hq
        p1 = next_5smooth(math.ceil((self.a + self.R) / hq1))
        p2 = next_5smooth(math.ceil((self.b + self.R) / hq2))
        return p1, p2

    @property
    def box_len(self) -> Tuple[float, float]:
        (p1, p2), (hq1, hq2) = self.box, self.hq
        return p1 * hq1, p2 * hq2

    def trapezoid_weights(self):
        """1D trapezoid weights (times the step) on the quadrature grid, both axes."""
        out = []
        for nq, hq in zip(self.nq, self.hq):
            w = np.full(nq + 1, hq)
            w[0] = w[-1] = 0.5 * hq
            out.append(w)
        return tuple(out)

    # Galerkin normalisers of the first two TBC rows (Section 3 after (ENUC11), App. A)
    def q_norm(self) -> np.ndarray:
        """q^(m,n) = ab/2 if m = 0 else ab/4, on the mode grid (row 1)."""
        q = np.full((self.M + 1, self.N + 1), self.a * self.b / 4.0)
        q[0, :] = self.a * self.b / 2.0
        return q

    def c_norm(self) -> np.ndarray:
        """c^(m,n) = ab/2 if n = 0 else ab/4, on the mode grid (row 2)."""
        cn = np.full((self.M + 1, self.N + 1), self.a * self.b / 4.0)
        cn[:, 0] = self.a * self.b / 2.0
        return cn
