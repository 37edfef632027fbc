"""Brute-force high-precision lattice step for tiny lattices (test
infrastructure only).

An independent second statement of the step, written against velocity
vectors rather than direction indices and evaluated with 40 significant
digits (mpmath), so FP64 rounding and summation order play no part. It follows the same equations
as the C oracle: moments and common velocity (Sec. II A), the Shan-Chen force
(Eq. (sc)), the force shift (Sec. II B), BGK towards Eq. (eqdis), pull
streaming with periodic wrap or a bounce-back wall at the z seam, and the
mass-conserving sink (Sec. II C). Solid wall nodes (Sec. III A, III B) hold
no fluid, reflect every population a fluid neighbour would pull from them,
and carry psi of given wall densities in the force. With one component
(ncomp=1, the multiphase form), the force takes the component itself as the
partner and the sink holds it at rho_H, booking what it removes.
"""
from __future__ import annotations

import itertools
import mpmath

mpmath.mp.dps = 40
mpf = mpmath.mpf

VELOCITIES = [e for e in itertools.product((-1, 0, 1), repeat=3) if sum(a * a for a in e) <= 2]
CS2 = mpf(1) / 3


def weight(e):
    n2 = sum(a * a for a in e)
    return mpf(1) / {0: 3, 1: 18, 2: 36}[n2]


def feq(e, rho, u):
    eu = sum(a * b for a, b in zip(e, u))
    uu = sum(a * a for a in u)
    return weight(e) * rho * (1 + eu / CS2 - uu / (2 * CS2) + eu * eu / (2 * CS2 * CS2))


def psi(rho, kind):
    if kind == "rho":
        return rho
    return 1 - mpmath.exp(-rho)


class ExactLattice:
    """State: populations[c][(x, y, z)][e] as mpf (post-stream, post-sink).

    Parameters given as strings or integers are converted exactly."""

    def __init__(self, nx, ny, nz, g, tau=(1, 1), psi_kind="rho", wall_z=False, sink=None, rho_h=0, solid=None,
                 wall_rho=(0, 0), ncomp=2):
        self.dims = (nx, ny, nz)
        self.g = mpf(g)
        self.tau = (mpf(tau[0]), mpf(tau[1]))
        self.psi_kind = psi_kind
        self.wall_z = wall_z
        self.sink = sink  # callable (x, y, z) -> bool, or None
        self.solid = solid  # callable (x, y, z) -> bool, or None
        self.wall_rho = (mpf(wall_rho[0]), mpf(wall_rho[1]))
        self.ncomp = ncomp
        self.rho_h = mpf(rho_h)
        self.evaporated = mpf(0)
        self.nodes = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]
        self.f = [dict(), dict()]

    def is_sink(self, node):
        return self.sink is not None and self.sink(*node) and not self.is_solid(node)

    def is_solid(self, node):
        return self.solid is not None and self.solid(*node)

    def _psi_field(self, rho):
        return [{n: psi(self.wall_rho[c] if self.is_solid(n) else rho[c][n], self.psi_kind) for n in self.nodes}
                for c in range(2)]

    def set_populations(self, pops):
        """pops[c][node][e] -> number; then the uncounted sink reset."""
        self.f = [{n: {e: (mpf(0) if self.is_solid(n) or c >= self.ncomp else mpf(v))
                       for e, v in pops[c][n].items()} for n in self.nodes} for c in range(2)]
        self._reset(count=False)

    def density(self, c, node):
        return sum(self.f[c][node].values())

    def _reset(self, count=True):
        if self.sink is None:
            return
        for n in self.nodes:
            if not self.is_sink(n):
                continue
            ra = self.density(0, n)
            rb = self.density(1, n)
            rbh = ra + rb - self.rho_h
            self.f[0][n] = {e: feq(e, self.rho_h, (0, 0, 0)) for e in VELOCITIES}
            if self.ncomp == 2:
                self.f[1][n] = {e: feq(e, rbh, (0, 0, 0)) for e in VELOCITIES}
            if count:
                self.evaporated += ra - self.rho_h

    def _neighbour_for_psi(self, node, e):
        nx, ny, nz = self.dims
        x, y, z = node
        zn = z + e[2]
        if zn < 0 or zn >= nz:
            zn = z if self.wall_z else zn % nz
        return ((x + e[0]) % nx, (y + e[1]) % ny, zn)

    def step(self):
        nx, ny, nz = self.dims
        rho = [{n: self.density(c, n) for n in self.nodes} for c in range(2)]
        ps = self._psi_field(rho)
        post = [dict(), dict()]
        for n in self.nodes:
            if self.is_solid(n):
                post[0][n] = {e: mpf(0) for e in VELOCITIES}
                post[1][n] = {e: mpf(0) for e in VELOCITIES}
                continue
            if self.is_sink(n):
                post[0][n] = dict(self.f[0][n])
                post[1][n] = dict(self.f[1][n])
                continue
            j = [[sum(self.f[c][n][e] * e[d] for e in VELOCITIES) for d in range(3)] for c in range(2)]
            force = []
            for c in range(2):
                s = [mpf(0)] * 3
                for e in VELOCITIES:
                    if e == (0, 0, 0):
                        continue
                    pn = ps[c if self.ncomp == 1 else 1 - c][self._neighbour_for_psi(n, e)]
                    for d in range(3):
                        s[d] += weight(e) * pn * e[d]
                force.append([-ps[c][n] * self.g * s[d] for d in range(3)])
            rt = rho[0][n] + rho[1][n]
            up = [(j[0][d] + j[1][d]) / rt for d in range(3)]
            for c in range(2):
                if c >= self.ncomp:
                    post[c][n] = {e: mpf(0) for e in VELOCITIES}
                    continue
                if rho[c][n] != 0:
                    u = [up[d] + self.tau[c] * force[c][d] / rho[c][n] for d in range(3)]
                else:
                    u = up
                post[c][n] = {e: self.f[c][n][e] - (self.f[c][n][e] - feq(e, rho[c][n], u)) / self.tau[c]
                              for e in VELOCITIES}
        new = [dict(), dict()]
        for n in self.nodes:
            x, y, z = n
            for c in range(2):
                new[c].setdefault(n, {})
            for e in VELOCITIES:
                zs = z - e[2]
                src = ((x - e[0]) % nx, (y - e[1]) % ny, zs % nz)
                for c in range(2):
                    if self.is_solid(n):
                        v = mpf(0)
                    elif (self.wall_z and (zs < 0 or zs >= nz)) or self.is_solid(src):
                        v = post[c][n][(-e[0], -e[1], -e[2])]
                    else:
                        v = post[c][src][e]
                    new[c][n][e] = v
        self.f = new
        self._reset(count=True)

    def velocity(self):
        """Barycentric velocity U of Eq. (velw) at every node of the state:
        U = (sum_c j^c + (F^A + F^B)/2) / (rho^A + rho^B), with the force of
        Eq. (sc) from the state's own densities; sink nodes feel no force
        (Sec. II C). Returns {node: (Ux, Uy, Uz)}."""
        rho = [{n: self.density(c, n) for n in self.nodes} for c in range(2)]
        ps = self._psi_field(rho)
        out = {}
        for n in self.nodes:
            if self.is_solid(n):
                out[n] = (mpf(0), mpf(0), mpf(0))
                continue
            num = [sum(self.f[c][n][e] * e[d] for c in range(2) for e in VELOCITIES) for d in range(3)]
            if not self.is_sink(n):
                for c in range(self.ncomp):
                    for e in VELOCITIES:
                        if e == (0, 0, 0):
                            continue
                        pn = ps[c if self.ncomp == 1 else 1 - c][self._neighbour_for_psi(n, e)]
                        for d in range(3):
                            num[d] += -ps[c][n] * self.g * weight(e) * pn * e[d] / 2
            rt = rho[0][n] + rho[1][n]
            out[n] = tuple(num[d] / rt for d in range(3))
        return out
