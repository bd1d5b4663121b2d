"""Seeded synthetic inputs for the implicit FLD radiation step.

This module only *generates inputs*: face coordinates, per-cell fields
(E_r, T_g, rho, kappa_R, kappa_P, c_v), boundary descriptions and dt.  It holds
none of the method's arithmetic (no metrics, no face coefficients, no solve);
the CPU oracle and the HIP library each derive everything else on their own.

The paper (Section 5.4.2) quotes no public dataset for the radiation solver, so
every workload here is synthetic, seeded with NumPy's PCG64 generator.  The
five workloads follow the shapes and value ranges of the paper's production
use (2D Cartesian and spherical-polar grids with stretched spacing, optically
thin to thick media, Section 3.2 and Section 5):

  c1  64x64 uniform Cartesian, Gaussian temperature bump, reflecting walls.
  c2  1024x1024 Cartesian stretched by 1.002 per cell, lognormal rho/T,
      Kramers opacity clipped to [1e-4, 1e4], Dirichlet (Marshak) x_lo side.
  c3  2048(r, log) x 512(theta) spherical-polar, power-law rho/T with 10 %
      angular modulation, inner flux, outer free-streaming, axis theta sides.
  c4  256 independent Cartesian blocks of uneven size with Dirichlet ghosts.
  c5  4096 x 2048 spherical-polar stress case, lognormal kappa (sigma_ln 4).

Every generator accepts smaller ``nx``/``ny`` so the same recipe can be used at
sizes a slow reference finishes in seconds.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

# Physical constants used only to build initial fields (E = a_R T^4) and the
# inner-boundary flux of the spherical workloads.  cgs units.
C_LIGHT = 2.99792458e10
SIGMA_SB = 5.670374419e-5
A_RAD = 4.0 * SIGMA_SB / C_LIGHT

# Boundary kinds (same numbering as the C enum ``fld_bc_kind``).
BC_REFLECT = 0
BC_DIRICHLET_FACE = 1
BC_DIRICHLET_GHOST = 2
BC_FLUX_IN = 3
BC_FREE_STREAM = 4
BC_AXIS = 5
BC_MILNE = 6

GEOM_CARTESIAN = 0
GEOM_SPHERICAL = 1

SIDES = ("xlo", "xhi", "ylo", "yhi")


@dataclasses.dataclass
class BC:
    kind: int = BC_REFLECT
    value: float = 0.0  # Dirichlet face: boundary temperature [K]; flux-in: F_in [erg cm^-2 s^-1]


@dataclasses.dataclass
class Problem:
    """One grid with its fields.  Arrays are float64, cell arrays shaped [ny, nx]."""

    name: str
    geom: int
    x_faces: np.ndarray  # nx+1 (x or r)
    y_faces: np.ndarray  # ny+1 (y or theta)
    E: np.ndarray
    T: np.ndarray
    rho: np.ndarray
    kappa_R: np.ndarray
    kappa_P: np.ndarray
    c_v: np.ndarray
    dt: float
    bc: List[BC]
    ghost_E: Optional[np.ndarray] = None  # Dirichlet-ghost values, packed xlo(ny) xhi(ny) ylo(nx) yhi(nx)
    nsteps: int = 1

    @property
    def nx(self) -> int:
        return self.x_faces.size - 1

    @property
    def ny(self) -> int:
        return self.y_faces.size - 1


@dataclasses.dataclass
class Batch:
    """Independent blocks solved together.  Fields are packed block after block."""

    name: str
    blocks: List[Problem]

    @property
    def nblocks(self) -> int:
        return len(self.blocks)

    def packed(self, field: str) -> np.ndarray:
        return np.concatenate([getattr(b, field).ravel() for b in self.blocks])

    def packed_ghosts(self) -> np.ndarray:
        return np.concatenate([b.ghost_E for b in self.blocks])


# ----------------------------------------------------------------------------
# random fields
# ----------------------------------------------------------------------------

def correlated_normal(shape, ell: float, seed: int) -> np.ndarray:
    """Unit-variance, zero-mean Gaussian random field on a periodic index grid.

    White noise N(0,1) is filtered in Fourier space by exp(-k^2 ell^2 / 4)
    (k in radians per cell), which gives the covariance exp(-d^2 / (2 ell^2)),
    then renormalised to zero mean and unit standard deviation.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(shape)
    ky = 2.0 * np.pi * np.fft.fftfreq(shape[0])
    kx = 2.0 * np.pi * np.fft.fftfreq(shape[1])
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    g = np.real(np.fft.ifft2(np.fft.fft2(w) * np.exp(-k2 * ell * ell / 4.0)))
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    return g


def lognormal(shape, median: float, sigma_ln: float, ell: float, seed: int) -> np.ndarray:
    return median * np.exp(sigma_ln * correlated_normal(shape, ell, seed))


def kramers(rho: np.ndarray, T: np.ndarray) -> np.ndarray:
    return 1e22 * rho * T ** -3.5


# ----------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------

def uniform_faces(n: int, d: float, x0: float = 0.0) -> np.ndarray:
    return x0 + d * np.arange(n + 1, dtype=np.float64)


def stretched_faces(n: int, d0: float, q: float) -> np.ndarray:
    widths = d0 * q ** np.arange(n, dtype=np.float64)
    return np.concatenate([[0.0], np.cumsum(widths)])


def log_faces(n: int, r0: float, r1: float) -> np.ndarray:
    return np.exp(np.linspace(np.log(r0), np.log(r1), n + 1))


def theta_faces(n: int) -> np.ndarray:
    f = np.linspace(0.0, np.pi, n + 1)
    f[0] = 0.0
    f[-1] = np.pi
    return f


def midpoints(f: np.ndarray) -> np.ndarray:
    return 0.5 * (f[1:] + f[:-1])


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def make_c1(nx: int = 64, ny: int = 64, seed: int = 1) -> Problem:
    d = 1e10
    xf, yf = uniform_faces(nx, d), uniform_faces(ny, d)
    xc, yc = midpoints(xf), midpoints(yf)
    X, Y = np.meshgrid(xc - 0.5 * xf[-1], yc - 0.5 * yf[-1])
    r2 = X * X + Y * Y
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(-1.0, 1.0, size=(ny, nx))
    T = 1e4 * (1.0 + 0.5 * np.exp(-r2 / (2.0 * (8.0 * d) ** 2))) * (1.0 + 1e-3 * u)
    shape = (ny, nx)
    return Problem(
        name="c1", geom=GEOM_CARTESIAN, x_faces=xf, y_faces=yf,
        E=A_RAD * T ** 4, T=T, rho=np.full(shape, 1e-9),
        kappa_R=np.ones(shape), kappa_P=np.ones(shape), c_v=np.full(shape, 1e8),
        dt=1e3, bc=[BC() for _ in range(4)])


def make_c2(nx: int = 1024, ny: int = 1024, seeds=(2, 3)) -> Problem:
    xf = stretched_faces(nx, 1e10, 1.002)
    yf = stretched_faces(ny, 1e10, 1.002)
    shape = (ny, nx)
    rho = lognormal(shape, 1e-9, 2.0, 32.0, seeds[0])
    T = lognormal(shape, 5e3, 1.0, 32.0, seeds[1])
    kap = np.clip(kramers(rho, T), 1e-4, 1e4)
    bc = [BC(BC_DIRICHLET_FACE, 2e4), BC(), BC(), BC()]
    return Problem(
        name="c2", geom=GEOM_CARTESIAN, x_faces=xf, y_faces=yf,
        E=A_RAD * T ** 4, T=T, rho=rho, kappa_R=kap, kappa_P=kap.copy(),
        c_v=np.full(shape, 1e8), dt=1e4, bc=bc)


def _spherical_rho_T(xf, yf, seed):
    rc, ny = midpoints(xf), yf.size - 1
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.uniform(-1.0, 1.0, size=ny)
    rho = 1e-8 * (rc[None, :] / 1e11) ** -2 * (1.0 + 0.1 * m[:, None])
    T = np.broadcast_to(1e4 * (rc[None, :] / 1e11) ** -0.5, rho.shape).copy()
    return rho, T


def _spherical_bc():
    return [BC(BC_FLUX_IN, SIGMA_SB * 1e4 ** 4), BC(BC_FREE_STREAM), BC(BC_AXIS), BC(BC_AXIS)]


def make_c3(nx: int = 2048, ny: int = 512, seed: int = 4) -> Problem:
    xf = log_faces(nx, 1e11, 1e14)
    yf = theta_faces(ny)
    rho, T = _spherical_rho_T(xf, yf, seed)
    kap = np.where(T < 1e4, 1e-3 * np.sqrt(rho) * T * T, kramers(rho, T))
    return Problem(
        name="c3", geom=GEOM_SPHERICAL, x_faces=xf, y_faces=yf,
        E=A_RAD * T ** 4, T=T, rho=rho, kappa_R=kap, kappa_P=kap.copy(),
        c_v=np.full(rho.shape, 1e8), dt=1e4, bc=_spherical_bc())


def make_c5(nx: int = 4096, ny: int = 2048, seeds=(4, 6), nsteps: int = 100) -> Problem:
    xf = log_faces(nx, 1e11, 1e14)
    yf = theta_faces(ny)
    rho, T = _spherical_rho_T(xf, yf, seeds[0])
    g = correlated_normal(rho.shape, 32.0, seeds[1])
    kap = np.clip(np.exp(4.0 * g), 1e-4, 1e4)
    return Problem(
        name="c5", geom=GEOM_SPHERICAL, x_faces=xf, y_faces=yf,
        E=A_RAD * T ** 4, T=T, rho=rho, kappa_R=kap, kappa_P=kap.copy(),
        c_v=np.full(rho.shape, 1e6), dt=1e5, bc=_spherical_bc(), nsteps=nsteps)


C4_SIDES = (16, 32, 48, 64, 96, 128)


def c4_block_shapes(nblocks: int = 256, seed: int = 5, sides=C4_SIDES):
    rng = np.random.Generator(np.random.PCG64(seed))
    nx = rng.choice(np.asarray(sides), size=nblocks)
    ny = rng.choice(np.asarray(sides), size=nblocks)
    return [(int(a), int(b)) for a, b in zip(nx, ny)]


def make_c4_block(b: int, nx: int, ny: int) -> Problem:
    d = 1e10
    shape = (ny, nx)
    ell = float(min(32, nx, ny))
    rho = lognormal(shape, 1e-9, 2.0, ell, 1000 + b)
    T = lognormal(shape, 5e3, 1.0, ell, 1000 + 10000 + b)
    kap = np.clip(kramers(rho, T), 1e-4, 1e4)
    # parent field: 2x coarser, covering the block plus its ghost ring
    py, px = (ny + 3) // 2, (nx + 3) // 2
    Tp = lognormal((py, px), 5e3, 1.0, 16.0, 2000 + b)
    J = np.arange(ny + 2) // 2
    I = np.arange(nx + 2) // 2
    Tring = Tp[J[:, None], I[None, :]]  # (ny+2, nx+2), index 0 and n+1 are ghosts
    ghostT = np.concatenate([
        Tring[1:ny + 1, 0], Tring[1:ny + 1, nx + 1],
        Tring[0, 1:nx + 1], Tring[ny + 1, 1:nx + 1]])
    bc = [BC(BC_DIRICHLET_GHOST) for _ in range(4)]
    return Problem(
        name=f"c4.{b}", geom=GEOM_CARTESIAN,
        x_faces=uniform_faces(nx, d), y_faces=uniform_faces(ny, d),
        E=A_RAD * T ** 4, T=T, rho=rho, kappa_R=kap, kappa_P=kap.copy(),
        c_v=np.full(shape, 1e8), dt=1e4, bc=bc, ghost_E=A_RAD * ghostT ** 4)


def make_c4(nblocks: int = 256, seed: int = 5, sides=C4_SIDES) -> Batch:
    shapes = c4_block_shapes(nblocks, seed, sides)
    return Batch("c4", [make_c4_block(b, nx, ny) for b, (nx, ny) in enumerate(shapes)])


MAKERS = {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4, "c5": make_c5}

# Full sizes of each workload (cells).
FULL_SIZES: Dict[str, tuple] = {"c1": (64, 64), "c2": (1024, 1024), "c3": (2048, 512), "c5": (4096, 2048)}


def make(name: str, **kw):
    return MAKERS[name](**kw)


def theta_slab(prob: Problem, j0: int, j1: int) -> Problem:
    """Rows j0 .. j1-1 of a spherical-polar problem at its own resolution: the
    share of one GPU if the grid were split into theta slabs.  A cut side is
    reflecting; a side on the pole keeps the axis."""
    ny = prob.ny
    if not (0 <= j0 < j1 <= ny):
        raise ValueError("slab rows out of range")
    rows = slice(j0, j1)
    bc = list(prob.bc)
    bc[2] = prob.bc[2] if j0 == 0 else BC()
    bc[3] = prob.bc[3] if j1 == ny else BC()
    return Problem(
        name=f"{prob.name}[{j0}:{j1}]", geom=prob.geom, x_faces=prob.x_faces.copy(),
        y_faces=prob.y_faces[j0:j1 + 1].copy(), E=prob.E[rows].copy(), T=prob.T[rows].copy(),
        rho=prob.rho[rows].copy(), kappa_R=prob.kappa_R[rows].copy(), kappa_P=prob.kappa_P[rows].copy(),
        c_v=prob.c_v[rows].copy(), dt=prob.dt, bc=bc, nsteps=prob.nsteps)
