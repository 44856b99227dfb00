"""Seeded synthetic inputs for the AAR stencil workloads.

This module holds random-number generation and input synthesis only:
right-hand sides, velocity fields, instance sizes and shifts, and the plain
description of each workload (grid, spacing, boundary conditions, stencil
radius, solver parameters).  None of the solver's arithmetic lives here: no
finite-difference weights, no operator, no preconditioner, no AAR step.  Both
the CPU oracle's tests and the GPU path draw their inputs from here, so the
two sides always see bit-identical data.

Random numbers come from a counter-based SplitMix64 (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): element i of
stream (seed, stream) is mix64(key + (i + 1) * 0x9E3779B97F4A7C15), where
key = mix64(seed * 0x9E3779B97F4A7C15 ^ (stream + 1) * 0xD1B54A32D192ED03).
Uniforms take the top 53 bits; normals use the Box-Muller transform on
consecutive pairs.

The paper's own workloads (electron densities and pseudocharges of aluminium
supercells for the Poisson equation, Eq. 8; the orbital-free DFT Helmholtz
kernel equation, Eq. 7; Matrix Market systems, Sec. 3.1) are not available.
The generators below stand in for them with the same structure: smooth
periodic charge distributions with zero mean, shifted periodic Helmholtz
operators, and nonsymmetric (upwinded convection-diffusion) operators.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_STREAM_MUL = 0xD1B54A32D192ED03
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

BC_ZERO_DIRICHLET = 0
BC_PERIODIC = 1


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _mix64_int(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    """64-bit key of stream `stream` under `seed`."""
    return _mix64_int((seed * 0x9E3779B97F4A7C15) ^ ((stream + 1) * _STREAM_MUL))


def splitmix64(key: int, count: int, start: int = 0) -> np.ndarray:
    """Counter-based SplitMix64 outputs for counters start+1 .. start+count."""
    with np.errstate(over="ignore"):
        ctr = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(key & _MASK64) + ctr * _GOLDEN
        return _mix64(z)


def uniform(seed: int, stream: int, count: int) -> np.ndarray:
    """U[0,1) doubles from the top 53 bits."""
    z = splitmix64(stream_key(seed, stream), count)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, stream: int, count: int) -> np.ndarray:
    """N(0,1) doubles by Box-Muller on consecutive uniform pairs."""
    pairs = (count + 1) // 2
    u = uniform(seed, stream, 2 * pairs)
    u1 = 1.0 - u[0::2]                      # (0, 1]: log is finite
    u2 = u[1::2]
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    out = np.empty(2 * pairs)
    out[0::2] = rad * np.cos(ang)
    out[1::2] = rad * np.sin(ang)
    return out[:count]


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """One linear system -a*Lap_h(u) + v.grad_h(u) + sigma*u = b on a 3D grid.

    Unknowns are stored with x fastest: index i + n0*(j + n1*k).  With zero
    Dirichlet boundaries grid point i sits at (i+1)*h; with periodic
    boundaries at i*h.  `radius` r selects the order-2r central second
    difference; `velocity` (planar [vx|vy|vz], radius 1 only) adds first-order
    upwind convection.
    """
    n: tuple
    h: tuple
    bc: tuple
    radius: int
    diffusion: float = 1.0
    shift: float = 0.0
    velocity: Optional[np.ndarray] = None

    @property
    def size(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


@dataclasses.dataclass
class Params:
    """AAR parameters: omega, beta (Eq. 3), history m (Eqs. 4-5), period p,
    tolerance on ||b - A x|| / ||b||, cap on iterations, precision mode."""
    omega: float = 0.6
    beta: float = 0.6
    m: int = 7
    p: int = 6
    tol: float = 1e-10
    max_iter: int = 1_000_000
    precision: int = 0          # 0 fp64, 1 mixed fp32, 2 mixed fp32 + bf16 history, 3/4 fp64 + fp32/bf16 history
    inner_tol: float = 0.0      # 0: the library's per-step rule
    max_outer: int = 30
    flags: int = 0


@dataclasses.dataclass
class Workload:
    name: str
    problems: list
    b: list
    x0: list
    params: Params


def dirichlet_poisson_problem(n: int) -> Problem:
    h = 1.0 / (n + 1)
    return Problem(n=(n, n, n), h=(h, h, h), bc=(BC_ZERO_DIRICHLET,) * 3, radius=1)


def dirichlet_poisson_7pt(n: int = 32, seed: int = 1, tol: float = 1e-8) -> Workload:
    """3D Poisson, 7-point, zero Dirichlet, h = 1/(n+1), b ~ N(0,1) i.i.d., x0 = 0."""
    prob = dirichlet_poisson_problem(n)
    b = normal(seed, 0, prob.size)
    return Workload(f"dirichlet_poisson_7pt_{n}^3", [prob], [b], [np.zeros(prob.size)],
                    Params(omega=0.6, beta=0.6, m=7, p=6, tol=tol))


def gaussian_charges(n: int, seed: int, count: int = 64, width_cells: float = 2.0) -> np.ndarray:
    """Sum of `count` Gaussian charges on the periodic unit cube minus its mean.

    Grid point i sits at i/n.  Charge q has centre c_q ~ U[0,1)^3, sign
    s_q = +-1 (fair coin) and width w = width_cells/n; its value at a point is
    s_q * exp(-d^2 / (2 w^2)) with d the minimum-image distance.  The sum is
    computed in FP64 and its FP64 mean is subtracted (a periodic Poisson
    right-hand side must integrate to zero).  This stands in for the
    electron-plus-pseudocharge density of the paper's periodic Poisson
    problem (Eq. 8).
    """
    u = uniform(seed, 1, 4 * count).reshape(count, 4)
    centres = u[:, :3]
    signs = np.where(u[:, 3] < 0.5, -1.0, 1.0)
    w = width_cells / n
    grid = np.arange(n) / n
    b = np.zeros((n, n, n))
    for q in range(count):
        prof = []
        for ax in range(3):
            d = grid - centres[q, ax]
            d -= np.round(d)                 # minimum image on the unit period
            prof.append(np.exp(-d * d / (2.0 * w * w)))
        # layout [k][j][i]: i (axis 0) fastest
        b += signs[q] * (prof[2][:, None, None] * prof[1][None, :, None] * prof[0][None, None, :])
    b -= b.mean()
    return b.reshape(-1)


def periodic_problem(n: int, radius: int, shift: float = 0.0) -> Problem:
    h = 1.0 / n
    return Problem(n=(n, n, n), h=(h, h, h), bc=(BC_PERIODIC,) * 3, radius=radius, shift=shift)


def periodic_poisson_charges(n: int = 192, seed: int = 2, radius: int = 6, tol: float = 1e-10,
                             precision: int = 0) -> Workload:
    """Periodic Poisson, order-2r central FD (37-point at r=6), Gaussian charges rhs."""
    prob = periodic_problem(n, radius)
    b = gaussian_charges(n, seed)
    return Workload(f"periodic_poisson_r{radius}_{n}^3", [prob], [b], [np.zeros(prob.size)],
                    Params(omega=0.6, beta=0.6, m=7, p=6, tol=tol, precision=precision))


def convection_field(n: int, seed: int, modes: int = 8, peclet: float = 0.5) -> np.ndarray:
    """Smooth random velocity on the Dirichlet grid, planar [vx|vy|vz].

    Component c is sum_q a_cq sin(2 pi k_cq . x + phi_cq) with a ~ N(0,1),
    k uniform over {-2..2}^3 minus the zero vector, phi ~ U[0, 2 pi).  The
    field is scaled so that the peak cell Peclet number max |v_c| h / 2
    (diffusion 1) equals `peclet`.  Points sit at (i+1) h, h = 1/(n+1).
    """
    h = 1.0 / (n + 1)
    kvecs = np.array([(a, b, c) for c in range(-2, 3) for b in range(-2, 3) for a in range(-2, 3)
                      if (a, b, c) != (0, 0, 0)], dtype=np.float64)
    amp = normal(seed, 2, 3 * modes).reshape(3, modes)
    pick = uniform(seed, 3, 3 * modes).reshape(3, modes)
    phase = 2.0 * np.pi * uniform(seed, 4, 3 * modes).reshape(3, modes)
    x = (np.arange(n) + 1.0) * h
    X = x[None, None, :]
    Y = x[None, :, None]
    Z = x[:, None, None]
    v = np.zeros((3, n, n, n))
    for c in range(3):
        for q in range(modes):
            kv = kvecs[min(int(pick[c, q] * len(kvecs)), len(kvecs) - 1)]
            v[c] += amp[c, q] * np.sin(2.0 * np.pi * (kv[0] * X + kv[1] * Y + kv[2] * Z) + phase[c, q])
    scale = peclet * 2.0 / (h * np.abs(v).max())
    return (v * scale).reshape(-1)


def convection_diffusion_upwind(n: int = 128, seed: int = 4, tol: float = 1e-10,
                                precision: int = 1) -> Workload:
    """-Lap u + v.grad u = b, 7-point + first-order upwind, zero Dirichlet, b ~ U(-1,1)."""
    prob = dirichlet_poisson_problem(n)
    prob.velocity = convection_field(n, seed)
    b = 2.0 * uniform(seed, 0, prob.size) - 1.0
    return Workload(f"convection_diffusion_upwind_{n}^3", [prob], [b], [np.zeros(prob.size)],
                    Params(omega=0.6, beta=0.6, m=10, p=4, tol=tol, precision=precision))


def batched_helmholtz(count: int = 512, seed: int = 5, nmin: int = 16, nmax: int = 96,
                      radius: int = 4, shift_max: float = 10.0, tol: float = 1e-10,
                      precision: int = 1, flags: int = 2) -> Workload:
    """`count` periodic shifted Helmholtz systems -Lap u + sigma u = b, order 2r.

    Edge n_i ~ U{nmin..nmax}, h_i = 1/n_i, sigma_i ~ U(0, shift_max),
    b_i ~ N(0,1) i.i.d.  A real, positive-shift stand-in for the paper's
    periodic Helmholtz problem (Eq. 7), which is solved many times over in
    the applications that motivate the method.  `flags` defaults to the
    solver's exact constant-mode deflation (value 2): small shifts make the
    constant vector a near-null mode that FP32 cannot resolve.
    """
    u = uniform(seed, 1, 2 * count).reshape(count, 2)
    probs, bs, xs = [], [], []
    for i in range(count):
        n = nmin + min(int(u[i, 0] * (nmax - nmin + 1)), nmax - nmin)
        sigma = shift_max * u[i, 1]
        if sigma == 0.0:
            sigma = shift_max * 2.0 ** -53
        prob = periodic_problem(n, radius, shift=sigma)
        probs.append(prob)
        bs.append(normal(seed, 100 + i, prob.size))
        xs.append(np.zeros(prob.size))
    return Workload(f"batched_helmholtz_r{radius}_{count}x[{nmin}..{nmax}]^3", probs, bs, xs,
                    Params(omega=0.6, beta=0.6, m=7, p=6, tol=tol, precision=precision, flags=flags))


# The periodic Helmholtz problem of orbital-free DFT (Sec. 3.2, Eq. 7):
# -(1/(4 pi)) Lap V + Q V = P rho^alpha with the paper's complex constants.
OFDFT_P = complex(0.003277, -0.009081)
OFDFT_Q = complex(-0.134992, -0.070225)
OFDFT_ALPHA = 5.0 / 6.0 + 5.0 ** 0.5 / 6.0


def ofdft_density(n: int, seed: int, lattice: float = 7.78, cells: int = 1, width: float = 0.9,
                  displacement: float = 0.15) -> np.ndarray:
    """Synthetic electron density on a periodic cube of `cells`^3 FCC cells of
    the given lattice constant (Bohr): one Gaussian per atom (width in Bohr,
    minimum-image distance), atoms displaced from the FCC sites by up to
    `displacement` of the lattice constant (uniform, seeded), on a floor of
    1e-3 so that rho^alpha is smooth; normalised to 3 electrons per atom.
    Stands in for the aluminium densities of the paper's Helmholtz problem."""
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    sites = np.array([(b + np.array([i, j, k])) / cells for i in range(cells) for j in range(cells)
                      for k in range(cells) for b in basis])
    u = uniform(seed, 2, sites.size).reshape(sites.shape)
    sites = (sites + displacement / cells * (2.0 * u - 1.0)) % 1.0
    L = lattice * cells
    grid = np.arange(n) / n
    rho = np.full((n, n, n), 1e-3)
    for c in sites:
        prof = []
        for ax in range(3):
            d = grid - c[ax]
            d -= np.round(d)
            prof.append(np.exp(-(d * L) ** 2 / (2.0 * width ** 2)))
        rho += prof[2][:, None, None] * prof[1][None, :, None] * prof[0][None, None, :]
    h = L / n
    rho *= 3.0 * len(sites) / (rho.sum() * h ** 3)
    return rho.reshape(-1)


def ofdft_helmholtz(n: int = 72, seed: int = 6, cells: int = 1, tol: float = 1e-10):
    """Complex periodic Helmholtz (Eq. 7): grid n^3 over `cells`^3 aluminium
    FCC cells (lattice 7.78 Bohr; n = 36 and 72 give the paper's h = 0.216
    and 0.108 Bohr for one cell), sixth-order central differences (r = 3),
    diffusion 1/(4 pi), complex shift Q, rhs P rho^alpha.  Returns
    (problem with the real part of Q as its shift, imaginary part of Q,
    complex rhs, Params)."""
    L = 7.78 * cells
    h = L / n
    prob = Problem(n=(n, n, n), h=(h, h, h), bc=(BC_PERIODIC,) * 3, radius=3, diffusion=1.0 / (4.0 * np.pi),
                   shift=OFDFT_Q.real)
    b = OFDFT_P * ofdft_density(n, seed, cells=cells) ** OFDFT_ALPHA
    return prob, OFDFT_Q.imag, b.astype(np.complex128), Params(omega=0.6, beta=0.6, m=7, p=6, tol=tol)


# ---- general sparse matrices (stand-ins for the nonsymmetric Matrix Market
# systems of Sec. 3.1, which are not available here) ----

@dataclasses.dataclass
class CsrMatrix:
    """A square matrix in compressed sparse rows: row i holds
    val[rowptr[i]:rowptr[i+1]] in columns col[...], strictly increasing,
    with the diagonal present."""
    rowptr: np.ndarray   # int64, n + 1
    col: np.ndarray      # int32, nnz
    val: np.ndarray      # float64, nnz

    @property
    def n(self) -> int:
        return len(self.rowptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        d[rows, self.col] = self.val
        return d


def _csr_from_bands(cols: np.ndarray, vals: np.ndarray, present: np.ndarray) -> CsrMatrix:
    """Rows from k bands given in increasing column order: cols, vals and
    present are (k, N) arrays; absent entries are dropped."""
    present = present.T
    counts = present.sum(axis=1)
    rowptr = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CsrMatrix(rowptr, cols.T[present].astype(np.int32), vals.T[present].astype(np.float64))


def reservoir_matrix(n: int = 16, seed: int = 7, log_sigma: float = 1.5, peclet: float = 0.5,
                     storage: float = 1e-2) -> CsrMatrix:
    """Single-phase flow through a heterogeneous medium on an n^3 grid (unit
    cube, h = 1/n, no-flow boundaries), the structure of the oil-reservoir
    matrices of the paper's sparse study: seven-point two-point-flux finite
    volumes with permeability K = exp(log_sigma g), g ~ N(0,1) per cell,
    face transmissibility 2 K_a K_b / (K_a + K_b) / h^2, first-order upwind
    convection by a smooth random velocity (peak cell Peclet `peclet` for unit
    permeability), and an accumulation term storage * mean(transmissibility)
    on the diagonal.  Nonsymmetric; every row strictly diagonally dominant."""
    N = n ** 3
    h = 1.0 / n
    K = np.exp(log_sigma * normal(seed, 1, N))
    vel = convection_field(n, seed + 100, peclet=peclet)
    idx = np.arange(N, dtype=np.int64)
    ii, jj, kk = idx % n, (idx // n) % n, idx // (n * n)
    coord = (ii, jj, kk)
    strides = (1, n, n * n)
    # bands in column order: -z, -y, -x, self, +x, +y, +z
    order = [(2, -1), (1, -1), (0, -1), None, (0, 1), (1, 1), (2, 1)]
    cols = np.zeros((7, N), dtype=np.int64)
    vals = np.zeros((7, N))
    present = np.zeros((7, N), dtype=bool)
    diag = np.zeros(N)
    tsum = 0.0
    tcount = 0
    for b, o in enumerate(order):
        if o is None:
            cols[b] = idx
            present[b] = True
            continue
        ax, d = o
        inside = (coord[ax] + d >= 0) & (coord[ax] + d < n)
        nb = np.where(inside, idx + d * strides[ax], idx)
        T = 2.0 * K * K[nb] / (K + K[nb]) / h ** 2
        T = np.where(inside, T, 0.0)
        cols[b] = nb
        present[b] = inside
        vals[b] -= T
        diag += T
        tsum += T.sum()
        tcount += int(inside.sum())
        # upwind: v > 0 takes the -axis neighbour, v < 0 the +axis one
        v = vel[ax]
        up = inside & ((v > 0) if d < 0 else (v < 0))
        vals[b] -= np.where(up, np.abs(v) / h, 0.0)
        diag += np.where(up, np.abs(v) / h, 0.0)
    diag += storage * tsum / max(tcount, 1)
    vals[3] = diag
    return _csr_from_bands(cols, vals, present)


def convection_matrix_2d(n: int = 64, peclet: float = 2.0) -> CsrMatrix:
    """-Lap u + v . grad u on an n x n grid (unit square, zero Dirichlet,
    h = 1/(n+1)) with centred differences for both terms and the rotating
    field v = c (sin(pi x) cos(pi y), -cos(pi x) sin(pi y)), c chosen for a
    peak cell Peclet number max |v_i| h / 2 = `peclet`.  Above Peclet 1 the off-diagonals change sign, so the matrix
    is no M-matrix: a hard nonsymmetric case of the kind the paper's fluid
    dynamics matrices are (Sec. 3.1)."""
    N = n * n
    h = 1.0 / (n + 1)
    idx = np.arange(N, dtype=np.int64)
    ii, jj = idx % n, idx // n
    x, y = (ii + 1) * h, (jj + 1) * h
    vx = np.sin(np.pi * x) * np.cos(np.pi * y)
    vy = -np.cos(np.pi * x) * np.sin(np.pi * y)
    scale = peclet * 2.0 / h / max(np.abs(vx).max(), np.abs(vy).max())
    vx, vy = vx * scale, vy * scale
    coord = (ii, jj)
    strides = (1, n)
    order = [(1, -1), (0, -1), None, (0, 1), (1, 1)]
    cols = np.zeros((5, N), dtype=np.int64)
    vals = np.zeros((5, N))
    present = np.zeros((5, N), dtype=bool)
    for b, o in enumerate(order):
        if o is None:
            cols[b] = idx
            vals[b] = 4.0 / h ** 2
            present[b] = True
            continue
        ax, d = o
        inside = (coord[ax] + d >= 0) & (coord[ax] + d < n)
        v = vx if ax == 0 else vy
        cols[b] = np.where(inside, idx + d * strides[ax], idx)
        vals[b] = -1.0 / h ** 2 + d * v / (2.0 * h)
        present[b] = inside
    return _csr_from_bands(cols, vals, present)


def workload(index: int, **kw) -> Workload:
    """The five evaluation workloads, 1-based, at full size unless overridden."""
    if index == 1:
        return dirichlet_poisson_7pt(**kw)
    if index == 2:
        return periodic_poisson_charges(**kw)
    if index == 3:
        kw.setdefault("n", 256)
        kw.setdefault("seed", 3)
        kw.setdefault("precision", 1)
        return periodic_poisson_charges(**kw)
    if index == 4:
        return convection_diffusion_upwind(**kw)
    if index == 5:
        return batched_helmholtz(**kw)
    raise ValueError(f"no workload {index}")


def random_vector(seed: int, stream: int, count: int) -> np.ndarray:
    """Plain N(0,1) test vector."""
    return normal(seed, stream, count)


def problem_size_bytes(prob: Problem, elem: int = 8) -> int:
    return prob.size * elem


__all__ = [
    "BC_ZERO_DIRICHLET", "BC_PERIODIC", "Problem", "Params", "Workload",
    "stream_key", "splitmix64", "uniform", "normal", "random_vector",
    "gaussian_charges", "convection_field",
    "dirichlet_poisson_problem", "periodic_problem",
    "dirichlet_poisson_7pt", "periodic_poisson_charges", "convection_diffusion_upwind",
    "batched_helmholtz", "workload",
]

