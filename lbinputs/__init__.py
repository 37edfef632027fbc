"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no lattice Boltzmann arithmetic: it only produces initial
density fields (and, for tests, random population sets) and the parameter sets
of the workloads. Both the oracle and the GPU library consume its output.

Workloads (the paper has no public dataset; every field here is synthetic):
  film     planar film, component A dense below ``z_film`` (Sec. III B setup)
  droplet  sphere of A centred in a cube, tanh profile of width 2
  sinus    small sinusoidal composition wave (Fick test, Sec. III A)
  batch64  64 cubic boxes, side log-uniform in [48, 160], seed 1
"""
from __future__ import annotations

import dataclasses

import numpy as np

_GOLDEN = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64(seed: int, k: np.ndarray) -> np.ndarray:
    """The k-th output (k = 0, 1, ...) of SplitMix64 seeded with ``seed``.

    SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the state advances by the
    golden-ratio increment and each output is a finalising mix of the state.
    Being counter-based, the k-th output needs no sequential state.
    """
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + (k + np.uint64(1)) * np.uint64(_GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, k: np.ndarray) -> np.ndarray:
    """Top 53 bits of the k-th SplitMix64 output divided by 2**53, in [0, 1)."""
    return (splitmix64(seed, k) >> np.uint64(11)).astype(np.float64) / float(1 << 53)


def node_noise(shape, amp: float, seed: int):
    """Per-node, per-component noise amp * (2u - 1) with u from draw 2*node + c."""
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.uint64)
    na = amp * (2.0 * uniform01(seed, 2 * idx) - 1.0)
    nb = amp * (2.0 * uniform01(seed, 2 * idx + 1) - 1.0)
    return na.reshape(shape), nb.reshape(shape)


def film(nx, ny, nz, z_film, rho_ma=0.7, rho_mi=0.04, noise=0.0, seed=0):
    """A dense (rho_ma) for z < z_film and rho_mi above; B the reverse."""
    z = np.arange(nz)[:, None, None]
    a = np.where(z < z_film, rho_ma, rho_mi) * np.ones((nz, ny, nx))
    b = (rho_ma + rho_mi) - a
    if noise:
        na, nb = node_noise(a.shape, noise, seed)
        a = a + na
        b = b + nb
    return a, b


def droplet(nx, ny, nz, radius, rho_in=0.7, rho_out=0.04, width=2.0, center=None):
    """rhoA(r) = (in+out)/2 - (in-out)/2 tanh((r-R)/width); B mirrored."""
    if center is None:
        center = ((nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2)
    z = np.arange(nz, dtype=np.float64)[:, None, None] - center[2]
    y = np.arange(ny, dtype=np.float64)[None, :, None] - center[1]
    x = np.arange(nx, dtype=np.float64)[None, None, :] - center[0]
    r = np.sqrt(x * x + y * y + z * z)
    a = 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * np.tanh((r - radius) / width)
    b = (rho_in + rho_out) - a
    return a, b


def sinus(nx, ny, nz, mean_a, mean_b, amp, modes=1):
    """A composition wave along z: rhoA = mean_a + amp sin(2 pi m z/nz), B opposite."""
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    s = np.sin(2 * np.pi * modes * z / nz) * np.ones((nz, ny, nx))
    return mean_a + amp * s, mean_b - amp * s


def random_populations(nx, ny, nz, seed, base_a=0.3, base_b=0.3, amp=0.02):
    """Random positive populations f[c, i, z, y, x]: w_i*base + amp*U(-1,1)/19."""
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    n = nx * ny * nz
    k = np.arange(2 * 19 * n, dtype=np.uint64)
    u = uniform01(seed, k).reshape(2, 19, nz, ny, nx)
    base = np.array([base_a, base_b])[:, None, None, None, None] * w[None, :, None, None, None]
    return base + amp * (2 * u - 1) / 19.0


# ---------------------------------------------------------------------------
# Workload definitions. Each is a plain dict of lattice and fluid parameters.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    steps: int
    g: float
    psi: str               # "rho" or "exp"
    sink: str              # "none", "zmax", "faces", "sphere"
    rho_h: float
    wall_z: bool
    init: str              # "film" or "droplet"
    init_args: dict
    sink_radius: float = 0.0
    phi_delta: tuple = (0.66, -0.66)
    # rho0^c of shifted storage (f - w_i rho0): the component's density in
    # the phase that fills most of the box (droplets: A's vapour, B's
    # liquid); films, whose two phases fill comparable volumes, take the
    # midpoint of the phases, which halves the largest stored deviation
    shift: tuple = (0.04, 0.70)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def densities(self):
        if self.init == "film":
            return film(self.nx, self.ny, self.nz, **self.init_args)
        if self.init == "droplet":
            return droplet(self.nx, self.ny, self.nz, **self.init_args)
        raise ValueError(self.init)


def film_small() -> Workload:
    """4x4x128 film: A (0.7) below z = 32, 0.04 above, B reversed; psi = rho,
    g = 0.9, tau = 1, sink rho_H = 0.04 on z = 127, wall below z = 0,
    1000 steps, 1e-4 noise from seed 0."""
    return Workload("film_4x4x128", 4, 4, 128, 1000, 0.9, "rho", "zmax", 0.04, True, "film",
                    dict(z_film=32, noise=1e-4, seed=0), shift=(0.37, 0.37))


def droplet_128() -> Workload:
    """128^3 droplet, radius 24, psi = rho, g = 0.9, sink rho_H = 0.04 on all faces."""
    return Workload("droplet_128^3", 128, 128, 128, 20000, 0.9, "rho", "faces", 0.04, False, "droplet",
                    dict(radius=24.0))


def film_deep() -> Workload:
    """64x64x512 film below z = 128, sink on z = 511, wall below z = 0."""
    return Workload("film_64x64x512", 64, 64, 512, 50000, 0.9, "rho", "zmax", 0.04, True, "film",
                    dict(z_film=128), shift=(0.37, 0.37))


def droplet_512() -> Workload:
    """512^3 droplet, radius 120, sink on all faces."""
    return Workload("droplet_512^3", 512, 512, 512, 5000, 0.9, "rho", "faces", 0.04, False, "droplet",
                    dict(radius=120.0))


def batch64(seed: int = 1):
    """64 droplet boxes: side L = rint(exp(U(ln 48, ln 160))), then rho_out in
    U[0.02, 0.06], then g in U[0.85, 1.0], each drawn 64 times in that order
    from numpy's default_rng(seed); radius 0.2 L; sink on all faces."""
    rng = np.random.default_rng(seed)
    side = np.rint(np.exp(rng.uniform(np.log(48), np.log(160), 64))).astype(int)
    rho_out = rng.uniform(0.02, 0.06, 64)
    g = rng.uniform(0.85, 1.0, 64)
    out = []
    for k in range(64):
        L = int(side[k])
        out.append(Workload(f"batch{k}_{L}^3", L, L, L, 10000, float(g[k]), "rho", "faces", float(rho_out[k]),
                            False, "droplet", dict(radius=0.2 * L)))
    return out


# Paper-parameter physics set: psi = 1 - exp(-rho), g = 3.6, tau = 1.
def paper_film(nz=128, z_film=64) -> Workload:
    """Film of Sec. III B: 4x4xnz, interface at z_film, wall at the bottom."""
    return Workload(f"paper_film_4x4x{nz}", 4, 4, nz, 20000, 3.6, "exp", "none", 0.04, True, "film",
                    dict(z_film=z_film))


def paper_droplet(n=64, radius=16.0, sink_radius=None, rho_h=0.02) -> Workload:
    """Droplet of Sec. III C at reduced size, spherical sink at R_H."""
    rh = sink_radius if sink_radius is not None else n / 2 - 1
    return Workload(f"paper_droplet_{n}^3", n, n, n, 20000, 3.6, "exp", "sphere", rho_h, False, "droplet",
                    dict(radius=radius), sink_radius=rh, phi_delta=(0.675, -0.675))
