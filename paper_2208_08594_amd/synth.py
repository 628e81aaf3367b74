"""Seeded synthetic reservoir Jacobians in BSR form.

This module only *generates inputs*: it holds none of the solver's arithmetic
and is shared, unchanged, by the CPU oracle tests and the GPU path.

The systems stand in for the fully implicit compositional Jacobians of the
paper (Sec. 2, block rows of n_c+1 equations per cell with pressure first) on
structured grids, since the SPE1/SPE5/SPE10 decks are not available:

* cell index  c = i + nx*(j + ny*k), 7-point stencil, block size b, pressure
  index p = 0 (the paper orders pressure first in every block row/column);
* two-point transmissibility with the harmonic mean of the cell
  permeabilities (the FVM flux of Sec. 2.2), unit geometry;
* off-diagonal block  A_cd = -T_cd * K  with  K = 1 e_p^T + eps (I - e_p e_p^T),
  eps = 0.1: every equation couples to the neighbour's pressure with weight
  T_cd and, weakly, to its own component;
* diagonal block  A_cc = a_c I + C_c + sum_d T_cd K, with accumulation a_c and a
  random coupling C_c (zero diagonal, entries U[-0.1, 0.1]);
* well cells carry a Dirichlet pressure row: row p of the block row is e_p^T in
  A_cc and zero in every A_cd (stored zeros are kept in the pattern);
* right-hand side U[-1, 1].

Draw order from ``numpy.random.default_rng(seed)``: log-permeability (n),
accumulation (n), coupling (n*b*b), rhs (n*b).  The layered/channelised
generator draws its own permeability fields first (see ``layered_logk``).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

EPS_COUPLING = 0.1


@dataclass
class BSRSystem:
    """A block-sparse system A x = rhs (BSR, row-major b x b blocks)."""

    name: str
    nx: int
    ny: int
    nz: int
    b: int
    p: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_ind: np.ndarray  # int32 [nnzb], strictly ascending per block row
    vals: np.ndarray  # float64 [nnzb, b, b]
    rhs: np.ndarray  # float64 [n*b]
    wells: np.ndarray  # int64 cell indices with a Dirichlet pressure row
    diag_pos: np.ndarray = field(repr=False, default=None)  # int64 [n]

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnzb(self) -> int:
        return int(self.col_ind.shape[0])

    @property
    def N(self) -> int:
        return self.n * self.b

    def dirichlet_row_mask(self) -> np.ndarray:
        """bool [nnzb, b]: True on the scalar rows that are Dirichlet well rows."""
        m = np.zeros((self.nnzb, self.b), dtype=bool)
        for c in self.wells:
            m[self.row_ptr[c]:self.row_ptr[c + 1], self.p] = True
        return m

    def to_dense(self) -> np.ndarray:
        n, b = self.n, self.b
        A = np.zeros((n * b, n * b))
        for c in range(n):
            for k in range(self.row_ptr[c], self.row_ptr[c + 1]):
                d = self.col_ind[k]
                A[c * b:(c + 1) * b, d * b:(d + 1) * b] = self.vals[k]
        return A


def _stencil(nx: int, ny: int, nz: int):
    """7-point pattern; returns row_ptr, col_ind, per-entry direction, diag_pos."""
    n = nx * ny * nz
    c = np.arange(n, dtype=np.int64)
    i = c % nx
    j = (c // nx) % ny
    k = c // (nx * ny)
    offs = np.array([-nx * ny, -nx, -1, 0, 1, nx, nx * ny], dtype=np.int64)
    exists = np.stack([k > 0, j > 0, i > 0, np.ones(n, bool),
                       i < nx - 1, j < ny - 1, k < nz - 1], axis=1)
    counts = exists.sum(1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    pos = row_ptr[:-1, None] + np.cumsum(exists, axis=1) - 1
    nnzb = int(row_ptr[-1])
    col_ind = np.empty(nnzb, dtype=np.int64)
    direction = np.empty(nnzb, dtype=np.int8)
    cols = c[:, None] + offs[None, :]
    col_ind[pos[exists]] = cols[exists]
    direction[pos[exists]] = np.broadcast_to(np.arange(7, dtype=np.int8), (n, 7))[exists]
    diag_pos = pos[:, 3].copy()
    return row_ptr, col_ind, direction, diag_pos


def _coupling_matrix(b: int, p: int) -> np.ndarray:
    K = np.zeros((b, b))
    K[:, p] = 1.0
    for r in range(b):
        if r != p:
            K[r, r] += EPS_COUPLING
    return K


def _harmonic(kc: np.ndarray, kd: np.ndarray) -> np.ndarray:
    return 2.0 * kc * kd / (kc + kd)


def assemble(name, nx, ny, nz, b, kh, kv, acc, rng, wells, p=0) -> BSRSystem:
    """Assemble the BSR Jacobian from cell permeabilities and accumulation.

    ``rng`` must already have produced the permeability and accumulation draws;
    the coupling (n*b*b) and rhs (n*b) are drawn here, in that order.
    """
    n = nx * ny * nz
    row_ptr, col_ind, direction, diag_pos = _stencil(nx, ny, nz)
    nnzb = col_ind.shape[0]
    C = rng.uniform(-0.1, 0.1, size=(n, b, b))
    idx = np.arange(b)
    C[:, idx, idx] = 0.0
    rhs = rng.uniform(-1.0, 1.0, size=n * b)

    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    off = direction != 3
    vertical = (direction == 0) | (direction == 6)
    T = np.zeros(nnzb)
    r_off, c_off = rows[off], col_ind[off]
    T_off = np.where(vertical[off], _harmonic(kv[r_off], kv[c_off]),
                     _harmonic(kh[r_off], kh[c_off]))
    T[off] = T_off
    Tsum = np.bincount(rows, weights=T, minlength=n)

    K = _coupling_matrix(b, p)
    vals = np.empty((nnzb, b, b))
    np.multiply(-T[:, None, None], K[None, :, :], out=vals)
    vals[diag_pos] = acc[:, None, None] * np.eye(b)[None] + C + Tsum[:, None, None] * K[None]

    wells = np.asarray(sorted(set(int(w) for w in wells)), dtype=np.int64)
    for c in wells:
        vals[row_ptr[c]:row_ptr[c + 1], p, :] = 0.0
        vals[diag_pos[c], p, p] = 1.0
    return BSRSystem(name=name, nx=nx, ny=ny, nz=nz, b=b, p=p,
                     row_ptr=row_ptr.astype(np.int32), col_ind=col_ind.astype(np.int32),
                     vals=vals, rhs=rhs, wells=wells, diag_pos=diag_pos)


def cell(nx, ny, i, j, k) -> int:
    return i + nx * (j + ny * k)


def corner_wells(nx, ny, nz):
    """Two wells at opposite corners (the small-case layout)."""
    return [cell(nx, ny, 0, 0, 0), cell(nx, ny, nx - 1, ny - 1, nz - 1)]


def lateral_corner_wells(nx, ny):
    """Four wells at the lateral corners of the top layer (k = 0)."""
    return [cell(nx, ny, 0, 0, 0), cell(nx, ny, nx - 1, 0, 0),
            cell(nx, ny, 0, ny - 1, 0), cell(nx, ny, nx - 1, ny - 1, 0)]


def lognormal_grid(nx, ny, nz, b, seed, sigma=1.0, kz_ratio=1.0, wells="corners2",
                   name=None) -> BSRSystem:
    """Lognormal permeability k = exp(N(0, sigma^2)); vertical k scaled by kz_ratio;
    accumulation U[0.5, 2]."""
    rng = np.random.default_rng(seed)
    n = nx * ny * nz
    logk = rng.normal(0.0, sigma, size=n)
    acc = rng.uniform(0.5, 2.0, size=n)
    kh = np.exp(logk)
    kv = kz_ratio * kh
    if wells == "corners2":
        w = corner_wells(nx, ny, nz)
    elif wells == "lateral4":
        w = lateral_corner_wells(nx, ny)
    elif wells == "none":
        w = []
    else:
        w = list(wells)
    return assemble(name or f"grid{nx}x{ny}x{nz}b{b}", nx, ny, nz, b, kh, kv, acc, rng, w)


def layered_logk(nx, ny, nz, rng):
    """log10 permeability of the heterogeneous layered case.

    Even layers: N(0, 1).  Odd layers: background N(-1.5, 0.75) crossed by
    y-aligned channel strips 4 cells wide every 12 cells (random x offset per
    layer) with log10 k ~ U[2, 3].  Clipped to [-3, 3] (1e-3 .. 1e3).
    Draws: n normals, nz integer offsets, n channel uniforms.
    """
    n = nx * ny * nz
    z = rng.normal(0.0, 1.0, size=n).reshape(nz, ny, nx)
    offsets = rng.integers(0, 12, size=nz)
    chan = rng.uniform(2.0, 3.0, size=n).reshape(nz, ny, nx)
    logk = z.copy()
    xs = np.arange(nx)
    for k in range(1, nz, 2):
        logk[k] = -1.5 + 0.75 * z[k]
        in_strip = ((xs - offsets[k]) % 12) < 4
        logk[k][:, in_strip] = chan[k][:, in_strip]
    return np.clip(logk, -3.0, 3.0).reshape(n)


def config(idx: int, seed: int = 0) -> BSRSystem:
    """The five synthetic workloads, by index.

    0: 10x10x10, b=4, lognormal sigma=1, 2 corner wells (4,000 unknowns)
    1: 64x64x32, b=4, lognormal sigma=1.5, kz/kh=0.1, 4 wells
    2: 128x128x64, b=7, as 1
    3: 60x220x85, b=4, layered channelised 1e-3..1e3, porosity U[0.05,0.3], 5 wells
    4: see ``serving_request``
    """
    if idx == 0:
        return lognormal_grid(10, 10, 10, 4, seed, 1.0, 1.0, "corners2", "cfg0_10x10x10_b4")
    if idx == 1:
        return lognormal_grid(64, 64, 32, 4, seed, 1.5, 0.1, "lateral4", "cfg1_64x64x32_b4")
    if idx == 2:
        return lognormal_grid(128, 128, 64, 7, seed, 1.5, 0.1, "lateral4", "cfg2_128x128x64_b7")
    if idx == 3:
        return layered_grid(60, 220, 85, 4, seed, "cfg3_60x220x85_b4")
    raise ValueError(f"no config {idx}")


def layered_grid(nx, ny, nz, b, seed, name=None) -> BSRSystem:
    """The heterogeneous layered/channelised case at any size: permeability
    from ``layered_logk``, k_z = 0.1 k_h, porosity U[0.05, 0.3] (accumulation
    phi / 0.175), wells at the four lateral corners and the centre of k = 0."""
    rng = np.random.default_rng(seed)
    logk = layered_logk(nx, ny, nz, rng)
    phi = rng.uniform(0.05, 0.3, size=nx * ny * nz)
    kh = 10.0 ** logk
    kv = 0.1 * kh
    acc = phi / 0.175
    w = lateral_corner_wells(nx, ny) + [cell(nx, ny, nx // 2, ny // 2, 0)]
    return assemble(name or f"layered_{nx}x{ny}x{nz}_b{b}", nx, ny, nz, b, kh, kv, acc, rng, w)


SERVING_SIDES = (16, 24, 32, 48, 64, 96)


def serving_request(r: int):
    """Shape of serving request r: (side, b), drawn from seed 1000 + r."""
    rng = np.random.default_rng(1000 + r)
    side = int(rng.choice(SERVING_SIDES))
    nc = int(rng.integers(2, 7))
    return side, nc + 1


def serving_system(r: int, side: int | None = None, b: int | None = None) -> BSRSystem:
    """First Newton step of serving request r (the small-case law on a cube)."""
    s, bb = serving_request(r)
    side = side or s
    b = b or bb
    return lognormal_grid(side, side, side, b, 1000 + r, 1.0, 1.0, "corners2",
                          f"req{r}_{side}^3_b{b}")


class DevicePatterns:
    """Device copies of the 7-point cube patterns (one per side), reused by
    every request of that side."""

    def __init__(self, device):
        self.device = device
        self._cache = {}

    def get(self, side):
        import torch
        if side not in self._cache:
            rp, ci, direction, diag_pos = _stencil(side, side, side)
            dev = self.device
            self._cache[side] = dict(
                row_ptr=torch.as_tensor(rp.astype(np.int32), device=dev),
                col_ind=torch.as_tensor(ci.astype(np.int32), device=dev),
                direction=torch.as_tensor(direction, device=dev),
                diag_pos=torch.as_tensor(diag_pos, device=dev),
                rows=torch.as_tensor(np.repeat(np.arange(len(rp) - 1), np.diff(rp)),
                                     device=dev))
        return self._cache[side]


def serving_system_device(r: int, side: int, b: int, patterns: "DevicePatterns", p: int = 0):
    """First Newton step of serving request r generated on the GPU with torch:
    the same law as serving_system (lognormal k with sigma 1, accumulation
    U[0.5, 2], coupling U[-0.1, 0.1] with zero diagonal, harmonic
    transmissibilities, two corner wells, rhs U[-1, 1]) drawn from a torch
    generator seeded with 1000 + r (other numbers than numpy's).  Serving
    requests up to 96^3 cells with b = 7 hold 2.4 GB of values, which is why
    they are drawn where they are solved.  Returns a dict of device tensors:
    row_ptr, col_ind (int32), vals (float64, nnzb*b*b), rhs (float64, n*b),
    keep (bool, nnzb*b*b: entries of the Dirichlet rows), and n, b, p."""
    import torch
    P = patterns.get(side)
    dev = patterns.device
    n = side ** 3
    gen = torch.Generator(device=dev)
    gen.manual_seed(1000 + r)
    f64 = torch.float64
    logk = torch.randn(n, generator=gen, device=dev, dtype=f64)
    acc = 0.5 + 1.5 * torch.rand(n, generator=gen, device=dev, dtype=f64)
    Cc = -0.1 + 0.2 * torch.rand((n, b, b), generator=gen, device=dev, dtype=f64)
    Cc.diagonal(dim1=1, dim2=2).zero_()
    rhs = 2.0 * torch.rand(n * b, generator=gen, device=dev, dtype=f64) - 1.0
    k = torch.exp(logk)
    rows, cols, direction = P["rows"], P["col_ind"].long(), P["direction"]
    off = direction != 3
    kr, kc = k[rows], k[cols]
    T = torch.where(off, 2.0 * kr * kc / (kr + kc), torch.zeros_like(kr))
    # per-cell sums in a fixed order (an index_add would use atomics)
    T7 = torch.zeros((n, 7), device=dev, dtype=f64)
    T7[rows, direction.long()] = T
    Tsum = T7.sum(dim=1)
    K = torch.zeros((b, b), device=dev, dtype=f64)
    K[:, p] = 1.0
    idx = torch.arange(b, device=dev)
    K[idx, idx] += torch.tensor([0.0 if q == p else EPS_COUPLING for q in range(b)],
                                device=dev, dtype=f64)
    vals = -T[:, None, None] * K[None]
    dpos = P["diag_pos"]
    vals[dpos] = acc[:, None, None] * torch.eye(b, device=dev, dtype=f64)[None] + Cc \
        + Tsum[:, None, None] * K[None]
    keep = torch.zeros(vals.shape, dtype=torch.bool, device=dev)
    rp = P["row_ptr"].long()
    for c in corner_wells(side, side, side):
        lo, hi = int(rp[c]), int(rp[c + 1])
        vals[lo:hi, p, :] = 0.0
        keep[lo:hi, p, :] = True
    for c in corner_wells(side, side, side):
        vals[dpos[c], p, p] = 1.0
    return dict(row_ptr=P["row_ptr"], col_ind=P["col_ind"], vals=vals.reshape(-1),
                rhs=rhs, keep=keep.reshape(-1), n=n, b=b, p=p)


def newton_step(sys: BSRSystem, step: int, seed: int) -> BSRSystem:
    """Next Newton step of a request: every stored scalar outside the Dirichlet
    rows is scaled by (1 + 0.05 u), u ~ U[-1, 1]; a fresh rhs is drawn."""
    rng = np.random.default_rng([seed, step])
    u = rng.uniform(-1.0, 1.0, size=sys.vals.shape)
    mask = sys.dirichlet_row_mask()[:, :, None]
    vals = np.where(mask, sys.vals, sys.vals * (1.0 + 0.05 * u))
    rhs = rng.uniform(-1.0, 1.0, size=sys.N)
    return BSRSystem(name=f"{sys.name}_s{step}", nx=sys.nx, ny=sys.ny, nz=sys.nz, b=sys.b,
                     p=sys.p, row_ptr=sys.row_ptr, col_ind=sys.col_ind, vals=vals, rhs=rhs,
                     wells=sys.wells, diag_pos=sys.diag_pos)


def poisson_csr(shape, seed=None):
    """Scalar 7-point (or 3-/5-point) Poisson matrix on a grid with Dirichlet
    boundary folded into the diagonal; returns (row_ptr, col_ind, vals)."""
    shape = tuple(shape)
    dims = len(shape)
    sizes = list(shape) + [1] * (3 - dims)
    nx, ny, nz = sizes
    row_ptr, col_ind, direction, diag_pos = _stencil(nx, ny, nz)
    vals = np.where(direction == 3, 2.0 * dims, -1.0)
    return row_ptr.astype(np.int32), col_ind.astype(np.int32), vals.astype(np.float64)


def random_bsr(n, b, density, seed, diag_boost=4.0, symmetric_pattern=False):
    """Random BSR matrix with a nonzero, boosted diagonal block in every row."""
    rng = np.random.default_rng(seed)
    pat = rng.random((n, n)) < density
    if symmetric_pattern:
        pat = pat | pat.T
    np.fill_diagonal(pat, True)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(pat.sum(1))
    col_ind = np.nonzero(pat)[1].astype(np.int32)
    vals = rng.uniform(-1.0, 1.0, size=(col_ind.shape[0], b, b))
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    dmask = rows == col_ind
    vals[dmask] += diag_boost * np.eye(b) * (1 + np.diff(row_ptr)[rows[dmask]])[:, None, None] / 2
    return row_ptr, col_ind, vals
