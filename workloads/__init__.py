"""Seeded synthetic inputs for the optimized-Schwarz NLS/GPE workloads.

This module is shared by the tests, the benchmark and the smoke check.  It
holds NO arithmetic of the method (no finite elements, no solves, no
transmission conditions): only the problem parameters of each workload and
seeded generators of the nodal input fields (initial datum u0, potential V,
strip widths, random initial interface vectors).  Both the CPU oracle and the
GPU library receive these arrays as plain inputs.

Problem statement (Section 2, eqs. Sch/BC/BCRobin):
    i u_t + c*Lap(u) + V u + beta*|u|^2 u = 0   on (xl,xr) x (yb,yu),
    Neumann on y = yb, yu;  d_n u - i*p_bc*u = 0 on x = xl, xr.
The Laplacian coefficient c is 1 for the cubic NLS and 1/2 for the GPE form
(Section 5.2, eq. GPE); V and beta carry the signs of eq. Sch.

Mesh convention: ncx x ncy CELLS, (ncx+1) x (ncy+1) nodes; node (i,k) sits at
(xl + i*hx, yb + k*hy); nodal arrays are x-major, y-fast: shape (ncx+1, ncy+1).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 1603_05110


@dataclass
class Problem:
    """The paper's problem statement for one instance (Sections 2-3)."""
    xl: float
    xr: float
    yb: float
    yu: float
    ncx: int
    ncy: int
    nsub: int
    strip_cells: List[int]
    lap_coef: float          # c: 1 (NLS) or 1/2 (GPE)
    beta: float              # f(u) = beta*|u|^2, sign as in eq. Sch
    p: float                 # Robin transmission parameter (S = -i p)
    p_bc: float              # Robin parameter on the physical x-edges (paper: = p)
    dt: float
    steps: int = 1
    name: str = ""
    # rotating-frame quadratic potential V(x,y) = vxx x^2 + vyy y^2 evaluated
    # at A(t) x~ (Section 5.2.1, eqs. x1Ax/u1u); omega = 0 means static V.
    omega: float = 0.0
    vxx: float = 0.0
    vyy: float = 0.0
    # transmission (and physical x-edge) condition: "robin" (S = -ip, eq.
    # TCSRobin) or "pade" (S_pade^m of eq. TCS with m terms and branch-cut
    # rotation theta, Section 2.1; the paper takes theta = pi/4)
    tc: str = "robin"
    pade_m: int = 0
    pade_theta: float = float(np.pi / 4)

    @property
    def hx(self) -> float:
        return (self.xr - self.xl) / self.ncx

    @property
    def hy(self) -> float:
        return (self.yu - self.yb) / self.ncy

    @property
    def nodes(self) -> int:
        return (self.ncx + 1) * (self.ncy + 1)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def node_coords(pb: Problem):
    """Node coordinates (x_i, y_k) as two 1-D arrays."""
    x = pb.xl + pb.hx * np.arange(pb.ncx + 1)
    y = pb.yb + pb.hy * np.arange(pb.ncy + 1)
    return x, y


def equal_strips(ncx: int, nsub: int) -> List[int]:
    if ncx % nsub:
        base = ncx // nsub
        cells = [base] * nsub
        for j in range(ncx - base * nsub):
            cells[j] += 1
        return cells
    return [ncx // nsub] * nsub


def uneven_strips(rng: np.random.Generator, ncx: int, nsub: int,
                  spread: float = 0.3, min_cells: int = 4) -> List[int]:
    """Strip widths of mean ncx/nsub perturbed by a uniform +-spread factor,
    rounded and fixed up so that they sum to ncx, each >= min_cells."""
    w = (ncx / nsub) * (1.0 + rng.uniform(-spread, spread, nsub))
    cells = np.maximum(np.round(w).astype(int), min_cells)
    diff = ncx - int(cells.sum())
    j = 0
    while diff != 0:
        step = 1 if diff > 0 else -1
        if cells[j % nsub] + step >= min_cells:
            cells[j % nsub] += step
            diff -= step
        j += 1
    return [int(c) for c in cells]


def dirichlet_strips(rng: np.random.Generator, ncx: int, nsub: int,
                     conc: float = 20.0, min_cells: int = 4) -> List[int]:
    """Uneven widths from Dirichlet(conc) proportions, >= min_cells each."""
    prop = rng.dirichlet(np.full(nsub, conc))
    free = ncx - min_cells * nsub
    raw = prop * free
    cells = np.floor(raw).astype(int)
    rem = free - int(cells.sum())
    order = np.argsort(-(raw - cells))
    cells[order[:rem]] += 1
    return [int(c) + min_cells for c in cells]


# --------------------------------------------------------------------------
# Initial data and potentials (nodal values)
# --------------------------------------------------------------------------

def gaussian_boost(pb: Problem, k: float = 1.0, a: float = 1.0) -> np.ndarray:
    """u0 = exp(-a(x^2+y^2)) * exp(i k x)."""
    x, y = node_coords(pb)
    X, Y = np.meshgrid(x, y, indexing="ij")
    return np.exp(-a * (X ** 2 + Y ** 2)) * np.exp(1j * k * X)


def trapezoid_norm2(pb: Problem, u: np.ndarray) -> float:
    """Trapezoidal-rule approximation of the integral of |u|^2 (input scaling
    only; not the finite-element mass)."""
    wx = np.full(pb.ncx + 1, pb.hx); wx[[0, -1]] *= 0.5
    wy = np.full(pb.ncy + 1, pb.hy); wy[[0, -1]] *= 0.5
    return float(np.einsum("i,k,ik->", wx, wy, np.abs(u) ** 2))


def normalised_gaussian_noise(pb: Problem, rng: np.random.Generator,
                              noise: float = 1e-3) -> np.ndarray:
    x, y = node_coords(pb)
    X, Y = np.meshgrid(x, y, indexing="ij")
    u = np.pi ** -0.5 * np.exp(-(X ** 2 + Y ** 2) / 2)
    u = u + noise * (rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape))
    return u / np.sqrt(trapezoid_norm2(pb, u))


def vortex_gaussian(pb: Problem, rng: np.random.Generator, nvort: int = 4,
                    radius: float = 2.0) -> np.ndarray:
    x, y = node_coords(pb)
    X, Y = np.meshgrid(x, y, indexing="ij")
    u = np.exp(-(X ** 2 + Y ** 2) / 2).astype(complex)
    for _ in range(nvort):
        r = radius * np.sqrt(rng.uniform())
        th = rng.uniform(0, 2 * np.pi)
        z = (X - r * np.cos(th)) + 1j * (Y - r * np.sin(th))
        u *= z / np.maximum(np.abs(z), 1e-300)
    return u / np.sqrt(trapezoid_norm2(pb, u))


def quadratic_potential(pb: Problem, axx: float, ayy: float) -> np.ndarray:
    x, y = node_coords(pb)
    X, Y = np.meshgrid(x, y, indexing="ij")
    return axx * X ** 2 + ayy * Y ** 2


def gaussian_bumps_potential(pb: Problem, rng: np.random.Generator, nb: int = 8,
                             amp: float = 5.0) -> np.ndarray:
    """Smooth random field: sum of nb Gaussians, rescaled to max|V| = amp."""
    x, y = node_coords(pb)
    X, Y = np.meshgrid(x, y, indexing="ij")
    V = np.zeros_like(X)
    for _ in range(nb):
        cx = rng.uniform(pb.xl, pb.xr)
        cy = rng.uniform(pb.yb, pb.yu)
        s = rng.uniform(1.0, 3.0)
        a = rng.uniform(-1.0, 1.0)
        V += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    return V * (amp / np.max(np.abs(V)))


def random_interface(rng: np.random.Generator, nsub: int, ny: int) -> np.ndarray:
    """Seeded complex normal interface vector, shape (2(N-1), ny)."""
    return (rng.standard_normal((2 * (nsub - 1), ny))
            + 1j * rng.standard_normal((2 * (nsub - 1), ny))) / np.sqrt(2)


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    problems: List[Problem]
    u0: List[np.ndarray]
    V: List[Optional[np.ndarray]]     # static nodal potential (None: rotating)
    algo: str = "classical"          # classical | precond
    label: str = ""
    extra: dict = field(default_factory=dict)


def rng_for(index: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + index + 1000 * salt))


def c1(ncells: int = 128) -> Workload:
    """Cubic NLS, V=0, (-10,10)^2, 2 x-strips, Robin p=1, dt=0.01, 20 steps."""
    pb = Problem(-10, 10, -10, 10, ncells, ncells, 2, equal_strips(ncells, 2),
                 lap_coef=1.0, beta=1.0, p=1.0, p_bc=1.0, dt=0.01, steps=20,
                 name=f"nls-{ncells}sq-2strips")
    u0 = gaussian_boost(pb, k=1.0)
    return Workload([pb], [u0], [np.zeros((ncells + 1, ncells + 1))],
                    algo="classical", label="C1")


def c2(ncells: int = 512, nsub: int = 16, steps: int = 200) -> Workload:
    """GPE, trap V=-(x^2+y^2)/2, beta=-50, (-8,8)^2, 16 strips, p=5, dt=1e-3."""
    pb = Problem(-8, 8, -8, 8, ncells, ncells, nsub, equal_strips(ncells, nsub),
                 lap_coef=0.5, beta=-50.0, p=5.0, p_bc=5.0, dt=1e-3, steps=steps,
                 name=f"gpe-trap-{ncells}sq-{nsub}strips")
    rng = rng_for(2)
    u0 = normalised_gaussian_noise(pb, rng)
    V = quadratic_potential(pb, -0.5, -0.5)
    return Workload([pb], [u0], [V], algo="precond", label="C2")


def c3(ninst: int = 64, steps: int = 100, sizes=(256, 384, 512, 768),
       nsub_range=(8, 32)) -> Workload:
    """Batch of independent cubic-NLS instances with uneven strips."""
    rng = rng_for(3)
    pbs, u0s, Vs = [], [], []
    for b in range(ninst):
        nb = int(rng.choice(sizes))
        nsub = int(rng.integers(nsub_range[0], nsub_range[1] + 1))
        cells = dirichlet_strips(rng, nb, nsub)
        p = float(rng.uniform(1.0, 10.0))
        pb = Problem(-10, 10, -10, 10, nb, nb, nsub, cells, lap_coef=1.0,
                     beta=1.0, p=p, p_bc=p, dt=0.01, steps=steps,
                     name=f"nls-batch-{b}-{nb}sq-{nsub}strips")
        Vs.append(gaussian_bumps_potential(pb, rng))
        u0s.append(gaussian_boost(pb, k=1.0))
        pbs.append(pb)
    return Workload(pbs, u0s, Vs, algo="classical", label="C3")


def c4_family(rng: np.random.Generator, ncells: int = 512, nsub: int = 16,
              steps: int = 200):
    """One member of the GPE family used to generate interface traces:
    V = -(x^2+y^2)/(2 w^2), w ~ U[0.5,2], beta ~ -U[10,200]."""
    w = float(rng.uniform(0.5, 2.0))
    beta = -float(rng.uniform(10.0, 200.0))
    pb = Problem(-8, 8, -8, 8, ncells, ncells, nsub, equal_strips(ncells, nsub),
                 lap_coef=0.5, beta=beta, p=5.0, p_bc=5.0, dt=1e-3, steps=steps,
                 name=f"gpe-family-w{w:.3f}-b{beta:.1f}")
    u0 = normalised_gaussian_noise(pb, rng)
    V = quadratic_potential(pb, -0.5 / w ** 2, -0.5 / w ** 2)
    return pb, u0, V


def c4(ncells: int = 1024, nsub: int = 32, steps: int = 500) -> Workload:
    rng = rng_for(4)
    pb, u0, V = c4_family(rng, ncells, nsub, steps)
    return Workload([pb], [u0], [V], algo="precond", label="C4")


def c5(ncells: int = 2048, nsub: int = 64, steps: int = 1000) -> Workload:
    """Rotating GPE solved in the rotating frame: V=-(x^2+1.2y^2)/2, beta=-500,
    omega=-0.7 in the sign convention of eq. GPE."""
    rng = rng_for(5)
    cells = uneven_strips(rng, ncells, nsub)
    pb = Problem(-16, 16, -16, 16, ncells, ncells, nsub, cells, lap_coef=0.5,
                 beta=-500.0, p=5.0, p_bc=5.0, dt=5e-4, steps=steps,
                 name=f"gpe-rot-{ncells}sq-{nsub}strips", omega=-0.7,
                 vxx=-0.5, vyy=-0.6)
    u0 = vortex_gaussian(pb, rng)
    return Workload([pb], [u0], [None], algo="precond", label="C5")


# --------------------------------------------------------------------------
# The paper's own experiments (Section 5)
# --------------------------------------------------------------------------

def nls_mesh1(nsub: int, p: float, steps: int = 50) -> Workload:
    """Section 5.1, first mesh: cubic NLS (V = 0, f(u) = |u|^2) on
    (-16,16) x (-8,8), dx = 1/128, dy = 1/8 (4096 x 128 cells, 4097 x 129
    nodes), N equal strips, Robin p on interfaces and physical x-edges,
    dt = 0.01, T = 0.5, u0 = exp(-x^2 - y^2 - 0.5 i x)."""
    ncx, ncy = 4096, 128
    pb = Problem(-16, 16, -8, 8, ncx, ncy, nsub, equal_strips(ncx, nsub), lap_coef=1.0,
                 beta=1.0, p=p, p_bc=p, dt=0.01, steps=steps,
                 name=f"nls-mesh1-{nsub}strips-p{p:g}")
    x, y = node_coords(pb)
    X, Y = np.meshgrid(x, y, indexing="ij")
    u0 = np.exp(-X ** 2 - Y ** 2 - 0.5j * X)
    return Workload([pb], [u0], [np.zeros((ncx + 1, ncy + 1))], algo="classical",
                    label="paper-5.1-mesh1")


def bec_1025(nsub: int, p: float = 180.0, steps: int = 1000) -> Workload:
    """Section 5.2.2, first mesh: rotating GPE on (-16,16)^2 with
    dx = dy = 1/32 (1024^2 cells), omega = 0.4, beta = 10.15, dt = 1e-4,
    T = 0.1 (1000 steps), u0 = pi^(-1/4) exp(-(x^2 + 2 y^2)/2), Robin p.
    The trap V = (gamma_x^2 x^2 + gamma_y^2 y^2)/2 is read with gamma_x = 1,
    gamma_y = 2 (u0 is the linear ground state of that trap), and the GPE of
    eq. GPE is put in the sign convention of eq. Sch: c = 1/2, V -> -V,
    beta -> -beta; solved in the rotating frame."""
    ncx = 1024
    pb = Problem(-16, 16, -16, 16, ncx, ncx, nsub, equal_strips(ncx, nsub), lap_coef=0.5,
                 beta=-10.15, p=p, p_bc=p, dt=1e-4, steps=steps,
                 name=f"bec-1025sq-{nsub}strips-p{p:g}", omega=0.4, vxx=-0.5, vyy=-2.0)
    x, y = node_coords(pb)
    X, Y = np.meshgrid(x, y, indexing="ij")
    u0 = (np.pi ** -0.25 * np.exp(-(X ** 2 + 2 * Y ** 2) / 2)).astype(complex)
    return Workload([pb], [u0], [None], algo="precond", label="paper-5.2.2-1025")


# --------------------------------------------------------------------------
# Learned interface guess: seeded initial parameters
# --------------------------------------------------------------------------

NET_SHAPES = [(64, 9, 5), (64,), (4, 64, 5), (4,)]


def net_init(seed: int) -> np.ndarray:
    """Initial parameters of the guess network, flat float32 in the order
    W1 (64,9,5), b1 (64), W2 (4,64,5), b2 (4): weights uniform in
    +-1/sqrt(fan_in), biases zero; the output layer is scaled by 0.1 so the
    untrained network predicts a small change."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 4000 + seed))
    w1 = rng.uniform(-1, 1, NET_SHAPES[0]) / np.sqrt(9 * 5)
    w2 = 0.1 * rng.uniform(-1, 1, NET_SHAPES[2]) / np.sqrt(64 * 5)
    parts = [w1, np.zeros(64), w2, np.zeros(4)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)
