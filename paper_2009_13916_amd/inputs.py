"""Seeded synthetic inputs for the MHFE-FV Darcy systems.

This module only draws random numbers and lays them out in the array
conventions of the C ABI (``include/edfa.h``): node lattice, per-cell
conductivity tensors, per-face boundary data, previous pressure.  It holds
none of the discretisation or solver arithmetic, so both the HIP path and
the CPU oracle can be fed from it.

The paper measures on four-layer SPE10 grids (Section 4), which are not
available here; these generators stand in for them with the same structure
classes: structured bricks with diagonal tensors, heterogeneous full tensors,
distorted hexahedra and strong channelised contrast.

Seeding: ``numpy.random.SeedSequence([13916, config_id]).spawn(6)`` gives,
in order, the streams for 0 permeability, 1 rotations/anisotropy,
2 node perturbation, 3 previous pressure / extra RHS, 4 observations,
5 batch sizes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Boundary-condition codes per face (must match include/edfa.h).
BC_NEUMANN = 0      # prescribed outward total face flux (0 = no flow); also interior faces
BC_DIRICHLET = 1    # prescribed face pressure


@dataclass
class Problem:
    """One MHFE-FV problem in C-ABI layout (all arrays host numpy)."""
    nx: int
    ny: int
    nz: int
    nodes: np.ndarray          # ((nx+1)(ny+1)(nz+1), 3) f64, i fastest
    K: np.ndarray              # (Ne, 6) f64: xx, yy, zz, xy, xz, yz
    c: np.ndarray              # (Ne,) f64 storage coefficient
    dt: float
    gamma: float
    bc_type: np.ndarray        # (Nf,) int8
    bc_value: np.ndarray       # (Nf,) f64
    p_prev: np.ndarray         # (Ne,) f64
    source: np.ndarray         # (Ne,) f64 (cell-mean source density)
    meta: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_faces(self) -> int:
        nx, ny, nz = self.nx, self.ny, self.nz
        return (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)


def seed_streams(config_id: int, extra: int | None = None):
    key = [13916, int(config_id)] if extra is None else [13916, int(config_id), int(extra)]
    return [np.random.default_rng(s) for s in np.random.SeedSequence(key).spawn(6)]


def brick_nodes(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0):
    x = np.linspace(0.0, lx, nx + 1)
    y = np.linspace(0.0, ly, ny + 1)
    z = np.linspace(0.0, lz, nz + 1)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)


def perturb_interior_nodes(nodes, nx, ny, nz, frac, rng):
    """Move every interior node by U(-frac, frac) * cell size per coordinate."""
    out = nodes.copy().reshape(nz + 1, ny + 1, nx + 1, 3)
    h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
    d = rng.uniform(-frac, frac, size=(nz - 1, ny - 1, nx - 1, 3)) * h
    out[1:-1, 1:-1, 1:-1, :] += d
    return out.reshape(-1, 3)


def x_dirichlet_faces(nx, ny, nz, p_left=1.0, p_right=0.0):
    """Dirichlet p on x=0 and x=1, no-flow elsewhere, in the face numbering of the ABI.

    x-faces come first, index ``i + (nx+1)*(j + ny*k)``.
    """
    nfx = (nx + 1) * ny * nz
    nf = nfx + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    bc_type = np.zeros(nf, dtype=np.int8)
    bc_val = np.zeros(nf, dtype=np.float64)
    j, k = np.meshgrid(np.arange(ny), np.arange(nz), indexing="ij")
    left = (0 + (nx + 1) * (j + ny * k)).ravel()
    right = (nx + (nx + 1) * (j + ny * k)).ravel()
    bc_type[left] = BC_DIRICHLET
    bc_type[right] = BC_DIRICHLET
    bc_val[left] = p_left
    bc_val[right] = p_right
    return bc_type, bc_val


def iso_tensor(k):
    K = np.zeros((k.size, 6))
    K[:, 0] = K[:, 1] = K[:, 2] = k
    return K


def diag_tensor(kx, ky, kz):
    K = np.zeros((kx.size, 6))
    K[:, 0], K[:, 1], K[:, 2] = kx, ky, kz
    return K


def haar_rotations(n, rng):
    """Uniform random rotations from normalised 4-Gaussian quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def pack_sym(M):
    """(n,3,3) symmetric -> (n,6) xx,yy,zz,xy,xz,yz."""
    return np.stack([M[:, 0, 0], M[:, 1, 1], M[:, 2, 2],
                     0.5 * (M[:, 0, 1] + M[:, 1, 0]),
                     0.5 * (M[:, 0, 2] + M[:, 2, 0]),
                     0.5 * (M[:, 1, 2] + M[:, 2, 1])], axis=1)


def gaussian_random_field(nx, ny, nz, corr_cells, sigma, rng):
    """Stationary field with covariance ~ exp(-r^2 / (2 l^2)), l in cells.

    White noise convolved (periodically) with a Gaussian kernel of standard
    deviation l/sqrt(2), then standardised and scaled to ``sigma``.
    Returned in cell order i fastest.
    """
    from scipy.ndimage import gaussian_filter
    w = rng.standard_normal((nz, ny, nx))
    f = gaussian_filter(w, sigma=corr_cells / np.sqrt(2.0), mode="wrap")
    f = (f - f.mean()) / f.std()
    return (sigma * f).ravel()


def channel_indicator(nx, ny, nz, rng, target_frac=0.30):
    """Binary sinuous channels along x until the channel volume reaches target_frac."""
    ind = np.zeros((nz, ny, nx), dtype=bool)
    xs = np.arange(nx) + 0.5
    yy = np.arange(ny)[None, :] + 0.5
    guard = 0
    while ind.mean() < target_frac and guard < 10000:
        guard += 1
        amp = rng.uniform(4, 16)
        lam = rng.uniform(32, 128)
        phase = rng.uniform(0, 2 * np.pi)
        y0 = rng.uniform(0, ny)
        width = rng.uniform(4, 10)
        thick = int(rng.integers(2, 5))
        z0 = int(rng.integers(0, max(1, nz - thick + 1)))
        yc = y0 + amp * np.sin(2 * np.pi * xs / lam + phase)          # (nx,)
        band = np.abs(yy - yc[:, None]) <= 0.5 * width                 # (nx, ny)
        ind[z0:z0 + thick, :, :] |= band.T[None, :, :]
    return ind.ravel(), float(ind.mean())


# --------------------------------------------------------------------------
# Workloads.  Shared physics: unit cube, Dirichlet p=1 at x=0 and p=0 at x=1,
# no flow elsewhere, porosity 0.2, total compressibility 1e-9 (c = 2e-10),
# gamma = 1, no source, previous pressure ~ U(0,1).
# --------------------------------------------------------------------------
PHI = 0.2
CT = 1e-9


def _common(nx, ny, nz, nodes, K, rngs, dt, meta):
    ne = nx * ny * nz
    bc_type, bc_val = x_dirichlet_faces(nx, ny, nz)
    p_prev = rngs[3].uniform(0.0, 1.0, ne)
    return Problem(nx, ny, nz, nodes, K, np.full(ne, PHI * CT), float(dt), 1.0,
                   bc_type, bc_val, p_prev, np.zeros(ne), meta)


def lognormal_iso_problem(n, sigma=1.0, config_id=1, dt=1.0, extra=None):
    """n^3 bricks, isotropic K with ln K ~ N(0, sigma^2) i.i.d. per cell (10^3 workload)."""
    rngs = seed_streams(config_id, extra)
    nx = ny = nz = int(n)
    k = np.exp(sigma * rngs[0].standard_normal(nx * ny * nz))
    return _common(nx, ny, nz, brick_nodes(nx, ny, nz), iso_tensor(k), rngs, dt,
                   {"workload": f"lognormal_iso_{nx}^3", "sigma_lnK": sigma})


def full_tensor_problem(nx, ny=None, nz=None, sigma=2.0, corr=8.0, config_id=2, dt=1.0):
    """Bricks with K = k1 R diag(1, a^-1/2, a^-1) R^T per cell (64^3 workload).

    R Haar-random per cell, a log-uniform in [10, 100], ln k1 a Gaussian
    random field (sigma, correlation length ``corr`` cells).
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    rngs = seed_streams(config_id)
    ne = nx * ny * nz
    lnk1 = gaussian_random_field(nx, ny, nz, corr, sigma, rngs[0])
    R = haar_rotations(ne, rngs[1])
    a = np.exp(rngs[1].uniform(np.log(10.0), np.log(100.0), ne))
    d = np.stack([np.ones(ne), a ** -0.5, 1.0 / a], axis=1) * np.exp(lnk1)[:, None]
    M = np.einsum("nij,nj,nkj->nik", R, d, R)
    return _common(nx, ny, nz, brick_nodes(nx, ny, nz), pack_sym(M), rngs, dt,
                   {"workload": f"full_tensor_grf_{nx}x{ny}x{nz}", "sigma_lnK": sigma,
                    "corr_cells": corr})


def channel_problem(nx=128, ny=128, nz=64, contrast=1e6, perturb=0.2, config_id=3, dt=1e-3):
    """Distorted hexahedra with binary sinuous channels (128x128x64 workload)."""
    rngs = seed_streams(config_id)
    nodes = perturb_interior_nodes(brick_nodes(nx, ny, nz), nx, ny, nz, perturb, rngs[2])
    ind, frac = channel_indicator(nx, ny, nz, rngs[0])
    k = np.where(ind, 1.0, 1.0 / contrast)
    return _common(nx, ny, nz, nodes, iso_tensor(k), rngs, dt,
                   {"workload": f"channel_{nx}x{ny}x{nz}", "channel_fraction": frac})


def anisotropic_problem(n=48, sigma=1.5, ratio=10.0, config_id=5, dt=1.0):
    """n^3 bricks, K = k diag(1, 1, 1/ratio), ln k ~ N(0, sigma^2) (48^3 adjoint workload)."""
    rngs = seed_streams(config_id)
    ne = n ** 3
    k = np.exp(sigma * rngs[0].standard_normal(ne))
    return _common(n, n, n, brick_nodes(n, n, n), diag_tensor(k, k, k / ratio), rngs, dt,
                   {"workload": f"anisotropic_{n}^3"})


def batch_problems(count=256, nmin=8, nmax=32, config_id=4):
    """Independent cubic grids, side ~ U{nmin..nmax}, sigma_lnK ~ U[0.5, 3]."""
    rng = seed_streams(config_id)[5]
    sides = rng.integers(nmin, nmax + 1, size=count)
    sigmas = rng.uniform(0.5, 3.0, size=count)
    return [lognormal_iso_problem(int(n), float(s), config_id=config_id, extra=i)
            for i, (n, s) in enumerate(zip(sides, sigmas))]


def observations(ne, count, rng):
    """Observation cells (without replacement) and target pressures ~ U(0,1)."""
    cells = np.sort(rng.choice(ne, size=count, replace=False)).astype(np.int64)
    return cells, rng.uniform(0.0, 1.0, size=count)
