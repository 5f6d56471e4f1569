"""Seeded synthetic inputs for the absorbing-boundary time stepper.

This module only *generates inputs*: grids of sample points, Gaussian wave
packets, Gaussian wells, harmonic-oscillator orbitals and the named workload
configurations.  It contains none of the method's arithmetic (no stencil, no
Dirichlet-to-Neumann map, no integrator), so both the HIP path and the FP64
oracle may draw their inputs from it without sharing any computation.

Array layout everywhere: ``[z][y][x]`` (x fastest) for one wavefunction and
``[z][y][x][orb]`` (orbital fastest) for a batch.  Grid points are
vertex-centred, ``x_j = (j - (n-1)/2) h``, so a box of ``n`` points per axis
spans ``[-(n-1)h/2, (n-1)h/2]`` (the paper's 3D test box [-1.5,1.5]^3 with
h = 0.1 has 31 points per axis, Sec. 4.2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


def axis_points(n: int, h: float) -> np.ndarray:
    """Vertex-centred sample points along one axis."""
    return (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * h


def mesh(shape: Tuple[int, int, int], h: float):
    """Return (Z, Y, X) coordinate arrays of shape ``shape = (nz, ny, nx)``."""
    nz, ny, nx = shape
    z, y, x = axis_points(nz, h), axis_points(ny, h), axis_points(nx, h)
    return np.meshgrid(z, y, x, indexing="ij")


def gaussian_packet(shape, h, center=(0.0, 0.0, 0.0), k=(0.0, 0.0, 0.0),
                    width=1.0, normalize=False) -> np.ndarray:
    """psi(x) = exp(-|x - c|^2 / (2 width^2)) exp(i k.x), complex128 [z][y][x].

    ``center`` and ``k`` are given as (x, y, z) triples.  With
    ``normalize=True`` the packet is scaled to h^3 sum |psi|^2 = 1.
    """
    Z, Y, X = mesh(shape, h)
    cx, cy, cz = center
    kx, ky, kz = k
    r2 = (X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2
    psi = np.exp(-r2 / (2.0 * width * width)) * np.exp(1j * (kx * X + ky * Y + kz * Z))
    if normalize:
        psi /= math.sqrt(h ** 3 * float(np.sum(np.abs(psi) ** 2)))
    return psi.astype(np.complex128)


def gaussian_well(shape, h, amplitude, center=(0.0, 0.0, 0.0), width=1.0) -> np.ndarray:
    """V(x) = -amplitude exp(-|x - c|^2 / (2 width^2)), float64 [z][y][x]."""
    Z, Y, X = mesh(shape, h)
    cx, cy, cz = center
    r2 = (X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2
    return (-amplitude * np.exp(-r2 / (2.0 * width * width))).astype(np.float64)


def random_complex(shape, seed, dtype=np.complex128) -> np.ndarray:
    """Uniform random complex field in the unit square, for operator parity."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=shape) + 1j * rng.uniform(-1.0, 1.0, size=shape)
    return a.astype(dtype)


def random_potential(shape, seed, scale=1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (scale * rng.uniform(-1.0, 1.0, size=shape)).astype(np.float64)


# --------------------------------------------------------------------------
# Harmonic-oscillator orbitals (TDHF-like batch)
# --------------------------------------------------------------------------

def _hermite_function(n: int, x: np.ndarray) -> np.ndarray:
    """Normalised 1D oscillator eigenfunction (omega = 1) by the stable
    three-term recurrence of Hermite functions."""
    h0 = np.pi ** -0.25 * np.exp(-0.5 * x * x)
    if n == 0:
        return h0
    h1 = math.sqrt(2.0) * x * h0
    for m in range(1, n):
        h0, h1 = h1, math.sqrt(2.0 / (m + 1)) * x * h1 - math.sqrt(m / (m + 1)) * h0
    return h1


def oscillator_quantum_numbers(count: int) -> List[Tuple[int, int, int]]:
    """The ``count`` lowest Cartesian states, ordered by shell n_x+n_y+n_z and
    then lexicographically."""
    out = []
    shell = 0
    while len(out) < count:
        for nx in range(shell, -1, -1):
            for ny in range(shell - nx, -1, -1):
                nz = shell - nx - ny
                out.append((nx, ny, nz))
        shell += 1
    return out[:count]


def oscillator_orbitals(shape, h, count, seed, kmax=2.0) -> np.ndarray:
    """``count`` oscillator eigenstates, each boosted by exp(i kappa n.x) with
    kappa ~ U[0, kmax] and n uniform on the sphere; returned as complex128
    ``[z][y][x][orb]`` normalised to h^3 sum |phi|^2 = 1 per orbital."""
    rng = np.random.default_rng(seed)
    Z, Y, X = mesh(shape, h)
    nz, ny, nx = shape
    ax, ay, az = axis_points(nx, h), axis_points(ny, h), axis_points(nz, h)
    out = np.empty(tuple(shape) + (count,), dtype=np.complex128)
    for j, (qx, qy, qz) in enumerate(oscillator_quantum_numbers(count)):
        base = (_hermite_function(qz, az)[:, None, None]
                * _hermite_function(qy, ay)[None, :, None]
                * _hermite_function(qx, ax)[None, None, :])
        kappa = rng.uniform(0.0, kmax)
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        phase = np.exp(1j * kappa * (v[0] * X + v[1] * Y + v[2] * Z))
        phi = base * phase
        phi /= math.sqrt(h ** 3 * float(np.sum(np.abs(phi) ** 2)))
        out[..., j] = phi
    return out


# --------------------------------------------------------------------------
# Named workloads (shapes, spacings, steps and seeded draws)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    n: int                      # interior points per axis (cubic box)
    h: float
    dt: float
    steps: int
    order: str                  # "dirichlet" | "periodic" | "zeroth" | "first"
    form: str                   # "box" | "faces"
    radius: int = 1
    s0: float = 1.0
    s1: float = 1.0
    s2: float = math.inf
    window: int = 0
    batch: int = 1
    meanfield: bool = False
    t0: float = 0.0
    t3: float = 0.0
    psi0: Optional[np.ndarray] = None
    V: Optional[np.ndarray] = None


def free_packet_small(n=32, h=0.25, steps=200, dt=0.005, radius=1, s0=1.0) -> Workload:
    """Free Gaussian packet, V = 0, exp(-|x-x0|^2/2) exp(2ix), x0 = box centre;
    zeroth-order condition in the dense box form."""
    shape = (n, n, n)
    psi0 = gaussian_packet(shape, h, center=(0.0, 0.0, 0.0), k=(2.0, 0.0, 0.0))
    return Workload("free_packet_32", n, h, dt, steps, "zeroth", "box", radius=radius,
                    s0=s0, psi0=psi0, V=np.zeros(shape))


def well_packet(n=128, h=0.2, steps=2000, dt=0.002, seed=2, radius=1, s1=1.0,
                window=0) -> Workload:
    """Single orbital in a static Gaussian well V = -5 exp(-|x|^2/2) plus a
    packet with k = (3, 1, 0) whose centre is drawn from U[-0.5, 0.5]^3;
    first-order condition."""
    rng = np.random.default_rng(seed)
    c = tuple(float(v) for v in rng.uniform(-0.5, 0.5, size=3))
    shape = (n, n, n)
    psi0 = gaussian_packet(shape, h, center=c, k=(3.0, 1.0, 0.0))
    V = gaussian_well(shape, h, 5.0)
    return Workload("well_packet_%d" % n, n, h, dt, steps, "first", "faces", radius=radius,
                    s1=s1, window=window, psi0=psi0, V=V)


def adjoint_packet(n=96, h=0.2, steps=500, dt=0.002, s1=1.0, window=0):
    """Adjoint workload parameters: well amplitude 5 at the origin, packet
    centred at x = 4 with k = (3, 0, 0) heading for the +x face; first order.
    Returns a dict of the scalar parameters (the fields are built from them,
    so that gradients can flow back to them)."""
    return {"n": n, "h": h, "steps": steps, "dt": dt, "s1": s1, "window": window,
            "amplitude": 5.0, "well_center": (0.0, 0.0, 0.0), "packet_center": (4.0, 0.0, 0.0),
            "k": (3.0, 0.0, 0.0)}


def uneven_batch(count=64, seed=4, sizes=(48, 64, 96, 128, 160), h=0.2, dt=0.002, steps=500):
    """Independent single-orbital instances: cubic box N drawn uniformly from
    ``sizes``, well amplitude ~ U[1, 5] centred ~ U[-1, 1]^3, packet centred
    ~ U[-1, 1]^3 with k ~ U[-3, 3]^3, order zeroth or first with probability
    1/2 each (local face operators, s = 1).  Returns a list of dicts with the
    box, the parameters and the fields."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        amp = float(rng.uniform(1.0, 5.0))
        wc = tuple(float(v) for v in rng.uniform(-1.0, 1.0, size=3))
        pc = tuple(float(v) for v in rng.uniform(-1.0, 1.0, size=3))
        k = tuple(float(v) for v in rng.uniform(-3.0, 3.0, size=3))
        order = "first" if rng.random() < 0.5 else "zeroth"
        shape = (n, n, n)
        out.append({"shape": shape, "h": h, "dt": dt, "steps": steps, "order": order, "s0": 1.0, "s1": 1.0,
                    "window": 0, "amplitude": amp, "well_center": wc, "packet_center": pc, "k": k,
                    "V": gaussian_well(shape, h, amp, center=wc),
                    "psi0": gaussian_packet(shape, h, center=pc, k=k)})
    return out
