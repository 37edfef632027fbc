"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it follows. None of them calls the GPU path.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import lbinputs as li
from oracle import analytic as an
from oracle import exact
from oracle.oracle import (PSI_EXP, PSI_RHO, SINK_FACES, SINK_NONE, SINK_SPHERE, SINK_ZMAX, Oracle,
                           OracleParams, feq, lattice_tables)


# ---------------------------------------------------------------------------
# Lattice and equilibrium (Sec. II A, Eq. (eqdis)): exact identities.
# ---------------------------------------------------------------------------

def test_d3q19_tables_exact_isotropy():
    ex, ey, ez, w, opp = lattice_tables()
    e = np.stack([ex, ey, ez], axis=1)
    W = [Fraction(x).limit_denominator(100) for x in w]
    assert W[0] == Fraction(1, 3) and all(x == Fraction(1, 18) for x in W[1:7])
    assert all(x == Fraction(1, 36) for x in W[7:])
    assert sum(W) == 1
    assert len({tuple(v) for v in e}) == 19
    for a in range(3):
        assert sum(W[i] * int(e[i, a]) for i in range(19)) == 0
        for b in range(3):
            s2 = sum(W[i] * int(e[i, a]) * int(e[i, b]) for i in range(19))
            assert s2 == (Fraction(1, 3) if a == b else 0)
            for c in range(3):
                assert sum(W[i] * int(e[i, a] * e[i, b] * e[i, c]) for i in range(19)) == 0
    # fourth-order isotropy: sum w e_a e_b e_c e_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc)/9
    for a, b, c, d in itertools.product(range(3), repeat=4):
        s4 = sum(W[i] * int(e[i, a] * e[i, b] * e[i, c] * e[i, d]) for i in range(19))
        iso = Fraction((a == b) * (c == d) + (a == c) * (b == d) + (a == d) * (b == c), 9)
        assert s4 == iso
    for i in range(19):
        assert np.all(e[opp[i]] == -e[i]) and opp[opp[i]] == i


def test_equilibrium_moments_closed_form():
    ex, ey, ez, w, opp = lattice_tables()
    e = np.stack([ex, ey, ez], axis=1).astype(float)
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho = rng.uniform(0.01, 1.0)
        u = rng.uniform(-0.1, 0.1, 3)
        f = feq(rho, u)
        assert abs(f.sum() - rho) < 1e-15
        assert np.allclose(f @ e, rho * u, atol=1e-16, rtol=0)
        P = (f[:, None, None] * e[:, :, None] * e[:, None, :]).sum(0)
        assert np.allclose(P, rho * (np.eye(3) / 3 + np.outer(u, u)), atol=1e-15, rtol=0)


# ---------------------------------------------------------------------------
# Special cases and invariants of the whole step.
# ---------------------------------------------------------------------------

def _params(nx, ny, nz, **kw):
    return OracleParams(nx, ny, nz, **kw)


@pytest.mark.parametrize("psi,g", [(PSI_RHO, 0.9), (PSI_EXP, 3.6)])
def test_uniform_rest_and_uniform_flow_are_fixed_points(psi, g):
    o = Oracle(_params(4, 3, 5, g=g, psi=psi))
    n = o.n
    u0 = np.array([0.03, -0.02, 0.01])
    f = np.zeros((2, 19, n))
    f[0] = feq(0.3, u0)[:, None]
    f[1] = feq(0.5, u0)[:, None]
    o.init_from_populations(f)
    o.step(10)
    out = o.populations().reshape(2, 19, n)
    assert np.max(np.abs(out - f)) < 1e-15
    # the Shan-Chen force of a uniform state vanishes (sum_i w_i e_i = 0)
    assert np.max(np.abs(o.total_force())) < 1e-13


@pytest.mark.parametrize("psi", [PSI_RHO, PSI_EXP])
def test_mass_and_momentum_conserved_periodic(psi):
    o = Oracle(_params(5, 4, 6, g=1.3, psi=psi))
    f = li.random_populations(5, 4, 6, seed=11)
    o.init_from_populations(f)
    d0 = o.diagnostics()
    o.step(40)
    d1 = o.diagnostics()
    for c in range(2):
        assert abs(d1["mass"][c] - d0["mass"][c]) <= 1e-13 * d0["mass"][c]
    # sum_x sum_c F^c = 0 for symmetric g, so total momentum is conserved
    assert np.max(np.abs(o.total_force())) < 1e-13
    assert np.max(np.abs(np.array(d1["momentum"]) - np.array(d0["momentum"]))) < 1e-13


@pytest.mark.parametrize("sink,wall,extra", [(SINK_ZMAX, True, {}), (SINK_FACES, False, {}),
                                             (SINK_SPHERE, False, {"sink_radius": 2.6})])
def test_sink_conserves_total_mass_and_books_evaporation(sink, wall, extra):
    """Sec. II C: the partner reset keeps each sink node's total density, so
    M^A + M^B is constant, and the mass of A removed equals E."""
    o = Oracle(_params(6, 6, 6, g=0.9, wall_z=wall, sink=sink, rho_h=0.02, **extra))
    a, b = li.droplet(6, 6, 6, 1.8)
    o.init_from_density(a, b)
    d0 = o.diagnostics()
    assert d0["evaporated"] == 0.0
    o.step(60)
    d1 = o.diagnostics()
    tot0 = d0["mass"][0] + d0["mass"][1]
    assert abs(d1["mass"][0] + d1["mass"][1] - tot0) <= 1e-13 * tot0
    assert abs(d1["mass"][0] + d1["evaporated"] - d0["mass"][0]) <= 1e-13 * tot0
    assert d1["evaporated"] > 0.0  # rho_H below the vapour density: evaporation


def test_sink_node_state_is_rest_equilibrium():
    o = Oracle(_params(4, 4, 8, g=0.9, wall_z=True, sink=SINK_ZMAX, rho_h=0.03))
    o.init_from_populations(li.random_populations(4, 4, 8, seed=5))
    o.step(3)
    f = o.populations()
    top = f[:, :, 7]
    fa = feq(0.03, (0, 0, 0))
    assert np.max(np.abs(top[0] - fa[:, None, None])) < 1e-17
    rb = top[1].sum(0)
    assert np.max(np.abs(top[1] - np.array(feq(1.0, (0, 0, 0)))[:, None, None] * rb[None])) < 1e-15


def _reflect(f, axis):
    """Mirror populations in one axis: node and direction components flip."""
    ex, ey, ez, w, opp = lattice_tables()
    e = np.stack([ex, ey, ez], axis=1)
    flip = e.copy()
    flip[:, axis] *= -1
    perm = [int(np.where((e == flip[i]).all(1))[0][0]) for i in range(19)]
    out = np.empty_like(f)
    sp_axis = {0: 3, 1: 2, 2: 1}[axis]  # axes of f[:, i]: (c, z, y, x)
    for i in range(19):
        out[:, perm[i]] = np.flip(f[:, i], axis=sp_axis)
    return out


@pytest.mark.parametrize("axis,sink,wall", [(0, SINK_ZMAX, True), (1, SINK_FACES, False), (2, SINK_FACES, False),
                                            (2, SINK_NONE, False)])
def test_mirror_symmetry(axis, sink, wall):
    """A mirrored initial state evolves into the mirrored state: catches wrong
    opposite directions, transposed axes and one-sided stencils."""
    p = _params(5, 4, 6, g=1.1, psi=PSI_EXP, wall_z=wall, sink=sink, rho_h=0.05)
    f0 = li.random_populations(5, 4, 6, seed=21)
    o1 = Oracle(p); o1.init_from_populations(f0); o1.step(7)
    o2 = Oracle(p); o2.init_from_populations(_reflect(f0, axis)); o2.step(7)
    assert np.max(np.abs(_reflect(o1.populations(), axis) - o2.populations())) < 1e-15


def test_component_exchange_symmetry():
    """Without a sink and with equal tau, swapping A and B commutes with a step."""
    p = _params(4, 5, 3, g=2.0, psi=PSI_EXP)
    f0 = li.random_populations(4, 5, 3, seed=8, base_a=0.2, base_b=0.6)
    o1 = Oracle(p); o1.init_from_populations(f0); o1.step(5)
    o2 = Oracle(p); o2.init_from_populations(f0[::-1].copy()); o2.step(5)
    assert np.max(np.abs(o1.populations()[::-1] - o2.populations())) < 1e-15


def test_planar_state_independent_of_cross_section():
    """A z-only state on 1x1xN and 3x2xN gives the same profiles."""
    a, b = li.film(1, 1, 24, 10)
    o1 = Oracle(_params(1, 1, 24, g=3.6, psi=PSI_EXP, wall_z=True, sink=SINK_ZMAX, rho_h=0.02))
    o1.init_from_density(a, b); o1.step(30)
    a3, b3 = li.film(3, 2, 24, 10)
    o3 = Oracle(_params(3, 2, 24, g=3.6, psi=PSI_EXP, wall_z=True, sink=SINK_ZMAX, rho_h=0.02))
    o3.init_from_density(a3, b3); o3.step(30)
    r1 = o1.density()[0][:, 0, 0]
    r3 = o3.density()[0]
    assert np.max(np.abs(r3 - r1[:, None, None])) < 1e-15


# ---------------------------------------------------------------------------
# Brute force in 40-digit arithmetic on tiny lattices.
# ---------------------------------------------------------------------------

def _to_exact_pops(f, nx, ny, nz):
    ex, ey, ez, w, opp = lattice_tables()
    pops = [dict(), dict()]
    for c in range(2):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    pops[c][(x, y, z)] = {(int(ex[i]), int(ey[i]), int(ez[i])): float(f[c, i, z, y, x])
                                          for i in range(19)}
    return pops


def _from_exact(lat, nx, ny, nz):
    ex, ey, ez, w, opp = lattice_tables()
    out = np.zeros((2, 19, nz, ny, nx))
    for c in range(2):
        for (x, y, z), d in lat.f[c].items():
            for i in range(19):
                out[c, i, z, y, x] = float(d[(int(ex[i]), int(ey[i]), int(ez[i]))])
    return out


@pytest.mark.parametrize("case", ["wall_zmax_rho", "periodic_exp", "unequal_tau", "sphere_rho", "solid_wall_exp",
                                  "one_component", "one_component_solid"])
def test_oracle_matches_exact_bruteforce(case):
    nx, ny, nz = 3, 2, 4
    kw = dict(g=0.9, psi=PSI_RHO, tau=(1.0, 1.0))
    ekw = dict(g="0.9", psi_kind="rho")
    steps = 3
    if case == "one_component":
        # the multiphase form: self-coupling -4.5, sink holding rho_H
        kw.update(ncomp=1, g=-4.5, psi=PSI_EXP, wall_z=True, sink=SINK_ZMAX, rho_h=0.125)
        ekw.update(ncomp=1, g="-4.5", psi_kind="exp", wall_z=True, sink=lambda x, y, z: z == nz - 1,
                   rho_h="0.125")
    if case == "one_component_solid":
        nz = 5
        kw.update(ncomp=1, g=-4.5, psi=PSI_EXP, solid_z=2, wall_rho=(0.5, 0.0), tau=(0.75, 1.0))
        ekw.update(ncomp=1, g="-4.5", psi_kind="exp", solid=lambda x, y, z: z < 2, wall_rho=("0.5", "0"),
                   tau=("0.75", "1"))
    if case == "solid_wall_exp":
        # solid wall of thickness 2 below the fluid and, through the periodic
        # wrap, above it; the wall carries psi(0.125), psi(0.25)
        nz = 5
        kw.update(g=2.0, psi=PSI_EXP, solid_z=2, wall_rho=(0.125, 0.25), sink=SINK_ZMAX, rho_h=0.03125)
        ekw.update(g="2.0", psi_kind="exp", solid=lambda x, y, z: z < 2, wall_rho=("0.125", "0.25"),
                   sink=lambda x, y, z: z == nz - 1, rho_h="0.03125")
    if case == "wall_zmax_rho":
        kw.update(wall_z=True, sink=SINK_ZMAX, rho_h=0.03125)
        ekw.update(wall_z=True, sink=lambda x, y, z: z == nz - 1, rho_h="0.03125")
    elif case == "periodic_exp":
        kw.update(g=3.6, psi=PSI_EXP)
        ekw.update(g="3.6", psi_kind="exp")
        steps = 2
    elif case == "unequal_tau":
        kw.update(tau=(0.75, 1.25))
        ekw.update(tau=("0.75", "1.25"))
    elif case == "sphere_rho":
        nx, ny, nz = 3, 3, 3
        kw.update(sink=SINK_SPHERE, sink_radius=1.2, rho_h=0.0625)
        ekw.update(sink=lambda x, y, z: (x - 1) ** 2 + (y - 1) ** 2 + (z - 1) ** 2 >= 1.44, rho_h="0.0625")
    f0 = li.random_populations(nx, ny, nz, seed=99, base_a=0.25, base_b=0.5, amp=0.05)
    o = Oracle(_params(nx, ny, nz, **kw))
    o.init_from_populations(f0)
    lat = exact.ExactLattice(nx, ny, nz, **ekw)
    lat.set_populations(_to_exact_pops(f0, nx, ny, nz))
    for _ in range(steps):
        o.step(1)
        lat.step()
    ref = _from_exact(lat, nx, ny, nz)
    got = o.populations()
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))
    assert abs(o.diagnostics()["evaporated"] - float(lat.evaporated)) < 1e-14
    # the barycentric velocity U of Eq. (velw), force term included; U is a
    # difference of momenta of the populations' size, which sets its
    # rounding scale where the flow is slow
    uref = np.zeros((3, nz, ny, nx))
    for (x, y, z), u in lat.velocity().items():
        for d in range(3):
            uref[d, z, y, x] = float(u[d])
    assert np.max(np.abs(o.velocity() - uref)) <= 1e-14 * max(np.max(np.abs(uref)), np.max(np.abs(ref)))


def test_velocity_of_uniform_moving_state_is_its_velocity():
    """A uniform state f^c = f^eq(rho^c, u0) feels no force, so U of Eq.
    (velw) is u0 at every node (to rounding)."""
    o = Oracle(_params(4, 3, 5, g=3.6, psi=PSI_EXP))
    u0 = np.array([0.031, -0.017, 0.009])
    f = np.zeros((2, 19, o.n))
    f[0] = feq(0.3, u0)[:, None]
    f[1] = feq(0.5, u0)[:, None]
    o.init_from_populations(f)
    U = o.velocity().reshape(3, -1)
    assert np.max(np.abs(U - u0[:, None])) < 1e-16


@pytest.mark.parametrize("wall", [False, True])
def test_velocity_force_term_closed_form(wall):
    """U of Eq. (velw) at rest populations is half the total Shan-Chen force
    over the total density. With rho^A = a uniform and rho^B = b + e sin(k z),
    psi = rho, the neighbour sum of Eq. (sc) is S^B_z = (1/18 + 4/36)
    (psi^B(z+1) - psi^B(z-1)) = (e/3) sin(k) cos(k z) and S^A = 0, so
    U_z = -g a (e/3) sin(k) cos(k z) / (2 (a + b + e sin(k z))), U_x = U_y = 0.
    Across a seam wall psi is mirrored, which changes only the end planes."""
    nz, a, b, e, g = 24, 0.3, 0.45, 0.02, 1.7
    o = Oracle(_params(2, 3, nz, g=g, psi=PSI_RHO, wall_z=wall))
    z = np.arange(nz, dtype=float)
    k = 2 * np.pi / nz
    rb = b + e * np.sin(k * z)
    o.init_from_density(np.full((nz, 3, 2), a), np.broadcast_to(rb[:, None, None], (nz, 3, 2)).copy())
    U = o.velocity()
    psi_up = np.roll(rb, -1)
    psi_dn = np.roll(rb, 1)
    if wall:
        psi_up[-1], psi_dn[0] = rb[-1], rb[0]
    expect = -g * a * (psi_up - psi_dn) / 6.0 / (2 * (a + rb))
    if not wall:   # the closed form of the periodic sine
        assert np.max(np.abs(expect + g * a * (e / 3) * np.sin(k) * np.cos(k * z) / (2 * (a + rb)))) < 1e-17
    assert np.max(np.abs(U[2] - expect[:, None, None])) < 1e-16
    assert np.max(np.abs(U[:2])) < 1e-17


# ---------------------------------------------------------------------------
# Solid walls of thickness 2 (Sec. III A, III B): bounce-back links out of
# solid nodes, psi of the wall densities in the force.
# ---------------------------------------------------------------------------

def test_solid_wall_without_force_equals_seam_wall():
    """With g = 0 the wall's psi plays no part, and a fluid above a solid
    layer of h planes streams exactly like the same fluid between seam walls:
    both reflect every link that leaves the fluid (half-way bounce-back)."""
    nx, ny, n, h = 3, 2, 7, 2
    f0 = li.random_populations(nx, ny, n, seed=31, base_a=0.3, base_b=0.4, amp=0.05)
    seam = Oracle(_params(nx, ny, n, g=0.0, wall_z=True, sink=SINK_ZMAX, rho_h=0.03))
    seam.init_from_populations(f0)
    solid = Oracle(_params(nx, ny, n + h, g=0.0, solid_z=h, wall_rho=(0.5, 0.5), sink=SINK_ZMAX, rho_h=0.03))
    fs = np.zeros((2, 19, n + h, ny, nx))
    fs[:, :, h:] = f0
    fs[:, :, :h] = 7.0          # anything put into the wall is cleared
    solid.init_from_populations(fs)
    seam.step(9)
    solid.step(9)
    got = solid.populations()
    assert np.array_equal(got[:, :, h:], seam.populations())
    assert not np.any(got[:, :, :h])
    ds, dw = solid.diagnostics(), seam.diagnostics()
    assert ds["mass"] == dw["mass"] and ds["evaporated"] == dw["evaporated"]


@pytest.mark.parametrize("psi", [PSI_RHO, PSI_EXP])
def test_solid_wall_conserves_each_mass(psi):
    o = Oracle(_params(4, 3, 9, g=1.7, psi=psi, solid_z=2, wall_rho=(0.2, 0.6)))
    o.init_from_populations(li.random_populations(4, 3, 9, seed=12))
    d0 = o.diagnostics()
    o.step(50)
    d1 = o.diagnostics()
    for c in range(2):
        assert abs(d1["mass"][c] - d0["mass"][c]) <= 1e-13 * d0["mass"][c]


@pytest.mark.parametrize("wall_rho", [(0.0, 0.0), (0.2, 0.55)])
def test_solid_wall_force_closed_form(wall_rho):
    """Uniform rest fluid (a, b) above a solid layer, psi = rho: at the first
    fluid plane the neighbour sum of Eq. (sc) has S^c_z = (1/18 + 4/36)
    (psi^c - psi^c_w) = (psi^c - psi^c_w)/6 (five links reach the wall), at
    the top plane (next to the wall through the periodic wrap) the opposite,
    and zero in between. U of Eq. (velw) is then
    U_z = -g (a S^B_z + b S^A_z) / (2 (a + b)); solid nodes report U = 0."""
    nz, h, a, b, g = 10, 2, 0.3, 0.45, 1.3
    o = Oracle(_params(2, 2, nz, g=g, psi=PSI_RHO, solid_z=h, wall_rho=wall_rho))
    o.init_from_density(np.full((nz, 2, 2), a), np.full((nz, 2, 2), b))
    U = o.velocity()
    s_a, s_b = (a - wall_rho[0]) / 6, (b - wall_rho[1]) / 6
    uz = -g * (a * s_b + b * s_a) / (2 * (a + b))
    expect = np.zeros(nz)
    expect[h], expect[nz - 1] = uz, -uz
    assert np.max(np.abs(U[2] - expect[:, None, None])) < 1e-16
    assert np.max(np.abs(U[:2])) < 1e-17
    ra, rb = o.density()
    assert not np.any(ra[:h]) and not np.any(rb[:h])


def test_solid_wall_planar_state_independent_of_cross_section():
    a, b = li.film(1, 1, 26, 12)
    kw = dict(g=3.6, psi=PSI_EXP, solid_z=2, wall_rho=(0.1, 0.0), sink=SINK_ZMAX, rho_h=0.02)
    o1 = Oracle(_params(1, 1, 26, **kw))
    o1.init_from_density(a, b); o1.step(30)
    a3, b3 = li.film(3, 2, 26, 12)
    o3 = Oracle(_params(3, 2, 26, **kw))
    o3.init_from_density(a3, b3); o3.step(30)
    assert np.max(np.abs(o3.density()[0] - o1.density()[0][:, :1, :1])) < 1e-15


def test_film_on_a_solid_wall_matches_printed_coexistence():
    """Sec. III B's film: 128 nodes, a solid wall of thickness 2 at the
    bottom that does not interact (psi_w = 0, "simple bounce back"), A (0.70)
    below the interface at 64 and B above (0.04 minority), psi = 1 -
    exp(-rho), g = 3.6. The bulk phases reach rho_ma ~ 0.704 and rho_mi ~
    0.036 (printed); measured 0.7092 and 0.0361. In a closed binary system
    the bulk point moves along the coexistence curve with what the wall
    layers adsorb: the seam wall gives 0.7080, a neutral solid wall (equal
    wall densities 0.37) 0.7113, so no wall rule reproduces 0.704 exactly."""
    nz = 128
    wall_rho = (0.0, 0.0)
    o = Oracle(_params(1, 1, nz, g=3.6, psi=PSI_EXP, solid_z=2, wall_rho=wall_rho))
    a, b = li.film(1, 1, nz, 64)
    o.init_from_density(a, b)
    o.step(60000)
    ra = o.density()[0][:, 0, 0]
    rho_ma, rho_mi = ra[20:44].mean(), ra[84:108].mean()
    print(f"wall_rho {wall_rho}: rho_ma = {rho_ma:.5f}, rho_mi = {rho_mi:.5f}, next to the wall "
          f"{ra[2]:.5f}, {ra[3]:.5f}")
    assert abs(rho_mi - 0.036) < 0.001, rho_mi
    assert abs(rho_ma - 0.704) < 0.006, rho_ma


@pytest.mark.parametrize("wall_rho", [(0.0, 0.7), (0.0, 0.0)])
def test_diffusion_into_bath_with_solid_wall(wall_rho):
    """Sec. III A with the wall as the paper places it: a solid layer of
    thickness 2 behind 125 fluid planes, the evaporation boundary
    (rho_H = 0.001) on the far fluid plane; the invading component follows the
    finite-difference Fick solution (a zero-flux mirror half a node before
    the first fluid plane) to 0.5 % of rho_H. A wall with the bath's
    densities exerts no force (measured 0.14 %). A wall that does not
    interact (psi_w = 0) leaves the bath's partner pulling the invading
    component towards it: the first fluid plane adsorbs an excess (4.7 % of
    rho_H), and beyond it the profile still follows Fick (0.21 %)."""
    nf, h, rho_h = 125, 2, 0.001
    o = Oracle(OracleParams(4, 4, nf + h, solid_z=h, wall_rho=wall_rho, g=3.6, psi=PSI_EXP, sink=SINK_ZMAX,
                            rho_h=rho_h))
    o.init_from_density(np.zeros((nf + h, 4, 4)), np.full((nf + h, 4, 4), 0.7))
    D = an.diffusion_small_gradient(0.5 * rho_h, 0.7, 3.6, "exp")
    T = 8000
    o.step(T)
    ra = o.density()[0][h:, 0, 0]
    dev = (ra - an.fick_bath_fd(nf, rho_h, D, T)) / rho_h
    if wall_rho[1] == 0.7:
        assert np.max(np.abs(dev)) < 0.005, np.max(np.abs(dev))
    else:
        assert np.max(np.abs(dev[1:])) < 0.005, np.max(np.abs(dev[1:]))
        assert 0.01 < dev[0] < 0.1, dev[0]


# ---------------------------------------------------------------------------
# The single-component multiphase form (Sec. I: the method carries over to the
# multiphase pseudopotential model).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("G", [-5.0, -6.0])
def test_one_component_coexistence_follows_equal_area_rule(G):
    """A planar liquid slab in its vapour (1 x 1 x 128, periodic) settles at
    the coexistence densities of the equal-area rule: measured within 0.6 %
    (vapour) and 0.05 % (liquid) at G = -5 and -6."""
    rv, rl = an.coexistence_single(G)
    nz = 128
    o = Oracle(_params(1, 1, nz, g=G, psi=PSI_EXP, ncomp=1, phi_delta=(rl, rv)))
    z = np.arange(nz)
    o.init_from_density(np.where((z >= 32) & (z < 96), rl, rv).astype(float).reshape(nz, 1, 1))
    m0 = o.diagnostics()["mass"][0]
    o.step(20000)
    r = o.density()[0][:, 0, 0]
    assert abs(r[0:16].mean() / rv - 1) < 0.01, (r[0:16].mean(), rv)
    assert abs(r[56:72].mean() / rl - 1) < 0.001, (r[56:72].mean(), rl)
    d = o.diagnostics()
    # FP64 rounding: 1e-13 of the mass per 10^3 steps
    assert abs(d["mass"][0] - m0) <= 2e-12 * m0 and d["mass"][1] == 0.0
    # the lower interface (density through the midpoint of the phases)
    # stays between nodes 31 and 32
    assert abs(d["z_interface"] - 31.5) < 0.6, d["z_interface"]


def test_one_component_evaporation_books_removed_mass():
    """The evaporation boundary on the single component: a liquid film on a
    solid wall with the top plane held below the vapour density; mass
    leaves through the boundary, M + E = M(0), and the film recedes."""
    G, nz = -5.0, 64
    rv, rl = an.coexistence_single(G)
    o = Oracle(_params(2, 2, nz, g=G, psi=PSI_EXP, ncomp=1, solid_z=2, wall_rho=(rl, 0.0), sink=SINK_ZMAX,
                       rho_h=0.5 * rv, phi_delta=(rl, rv)))
    z = np.arange(nz)
    o.init_from_density(np.broadcast_to(np.where(z < 32, rl, rv).reshape(nz, 1, 1), (nz, 2, 2)).copy())
    d0 = o.diagnostics()
    o.step(3000)
    d1 = o.diagnostics()
    assert d1["evaporated"] > 0
    assert abs(d1["mass"][0] + d1["evaporated"] - d0["mass"][0]) <= 1e-12 * d0["mass"][0]
    assert d1["z_interface"] < d0["z_interface"]


# ---------------------------------------------------------------------------
# Fick's law with the analytic coefficient (Sec. III A).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mean,g,psi,tau", [
    (0.37, 0.9, "rho", 1.0),    # the configs' fluid at the symmetric composition
    (0.30, 1.2, "exp", 1.0),    # psi = 1 - exp(-rho)
    (0.35, 0.0, "rho", 0.8),    # ideal mixing: D = c_s^2 (tau - 1/2)
])
def test_sinusoid_decays_with_paper_diffusion_coefficient(mean, g, psi, tau):
    """A composition wave decays as exp(-D k^2 t) with D of the small-gradient
    formula. At a symmetric composition the paper's assumption
    grad rho^B = -grad rho^A holds exactly, so the match is tight."""
    nz = 128
    o = Oracle(_params(1, 1, nz, g=g, psi=PSI_RHO if psi == "rho" else PSI_EXP, tau=(tau, tau)))
    a, b = li.sinus(1, 1, nz, mean, mean, 1e-5)
    o.init_from_density(a, b)
    s = np.sin(2 * np.pi * np.arange(nz) / nz)
    amps, ts = [], []
    for k in range(9):
        if k:
            o.step(500)
        ra, _ = o.density()
        amps.append((ra[:, 0, 0] - mean) @ s / (s @ s))
        ts.append(500 * k)
    slope = np.polyfit(ts[2:], np.log(amps[2:]), 1)[0]
    d_meas = -slope / (2 * np.pi / nz) ** 2
    d_paper = an.diffusion_small_gradient(mean, mean, g, psi, tau)
    assert abs(d_meas / d_paper - 1) < 0.01, (d_meas, d_paper)


def test_diffusion_into_bath_follows_ficks_law():
    """Sec. III A diffusion test: a box filled with the partner component
    (rho = 0.7, g = 3.6, psi = 1 - exp(-rho)), a wall at one end and an
    evaporation boundary holding the diffusing component at rho_H = 0.001 at
    the other; the component invades the box as Fick's second law (Eq.
    (fick2)) with the coefficient of Eq. (diffu-t-1) predicts. The reference
    is an explicit finite-difference solution on the same nodes: the
    boundary node held at rho_H, a zero-flux mirror half a node beyond z = 0
    (the half-way bounce-back wall), the partner's gradient negligible."""
    nz, rho_h = 125, 0.001
    o = Oracle(OracleParams(4, 4, nz, wall_z=True, g=3.6, psi=PSI_EXP, sink=SINK_ZMAX, rho_h=rho_h))
    o.init_from_density(np.zeros((nz, 4, 4)), np.full((nz, 4, 4), 0.7))
    D = an.diffusion_small_gradient(0.5 * rho_h, 0.7, 3.6, "exp")
    T = 8000
    u = an.fick_bath_fd(nz, rho_h, D, T)
    o.step(T)
    ra = o.density()[0]
    assert np.ptp(ra, axis=(1, 2)).max() < 1e-15   # planar
    err = np.max(np.abs(ra[:, 0, 0] - u)) / rho_h
    assert err < 0.005, err   # measured 0.14 % of rho_H
    assert u[nz // 2] > 0.05 * rho_h   # the front has crossed half the box


# ---------------------------------------------------------------------------
# Diagnostics on constructed fields (x_I of Sec. III B, R_I of Sec. III C).
# ---------------------------------------------------------------------------

def test_interface_height_is_the_zero_of_a_linear_profile():
    """x_I is the first zero of the plane mean of rhoA - rhoB scanning up from
    z = 0, linearly interpolated: exact for a profile linear in z (here with a
    cross-section whose plane mean, not each node, is linear)."""
    nx, ny, nz, zs = 3, 2, 48, 20.3
    z = np.arange(nz, dtype=float)[:, None, None]
    wob = 0.004 * np.array([[1.0, -1.0, 0.5], [-0.5, 0.0, 0.0]])[None]   # zero mean over the plane
    a = 0.37 - 0.01 * (z - zs) + wob + np.zeros((nz, ny, nx))
    b = 0.37 + 0.01 * (z - zs) - wob + np.zeros((nz, ny, nx))
    o = Oracle(_params(nx, ny, nz))
    o.init_from_density(a, b)
    assert abs(o.diagnostics()["z_interface"] - zs) < 1e-12


def test_droplet_radius_of_a_sharp_droplet():
    """R_I = (3 sum(phi) / 4 pi)^(1/3) with phi = clamp((rhoA - rhoB -
    D_out) / (D_in - D_out), 0, 1): a droplet of bulk densities inside radius
    R gives phi = 1 on its nodes and 0 elsewhere, so R_I is the radius of a
    sphere of their count (brute force)."""
    n, R = 24, 7.3
    c = (n - 1) / 2
    zz, yy, xx = np.meshgrid(*(np.arange(n) - c,) * 3, indexing="ij")
    inside = xx ** 2 + yy ** 2 + zz ** 2 < R * R
    a = np.where(inside, 0.70, 0.04)
    b = np.where(inside, 0.04, 0.70)
    o = Oracle(_params(n, n, n, phi_delta=(0.66, -0.66)))
    o.init_from_density(a, b)
    expect = (3 * inside.sum() / (4 * np.pi)) ** (1 / 3)
    assert abs(o.diagnostics()["r_droplet"] - expect) < 1e-12
    # halfway densities count half a node each
    a2 = np.where(inside, 0.37, 0.04)
    b2 = np.where(inside, 0.37, 0.70)
    o.init_from_density(a2, b2)
    assert abs(o.diagnostics()["r_droplet"] - (3 * 0.5 * inside.sum() / (4 * np.pi)) ** (1 / 3)) < 1e-12


# ---------------------------------------------------------------------------
# Planar film (Sec. III B): coexistence and the sqrt(t) law.
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def equilibrated_film64():
    nz = 64
    o = Oracle(_params(1, 1, nz, g=3.6, psi=PSI_EXP, wall_z=True))
    a, b = li.film(1, 1, nz, nz // 2)
    o.init_from_density(a, b)
    o.step(40000)
    return o.populations().copy()


def test_film_coexistence_matches_printed_values():
    """Sec. III B: after equilibration rho_ma ~ 0.704, rho_mi ~ 0.036 and an
    interface about 5 nodes wide (psi = 1 - exp(-rho), g = 3.6, tau = 1)."""
    nz = 128
    o = Oracle(_params(1, 1, nz, g=3.6, psi=PSI_EXP, wall_z=True))
    a, b = li.film(1, 1, nz, 64)
    o.init_from_density(a, b)
    o.step(60000)
    ra = o.density()[0][:, 0, 0]
    rho_ma, rho_mi = ra[20:44].mean(), ra[84:108].mean()
    assert abs(rho_mi - 0.036) < 0.001, rho_mi
    assert abs(rho_ma - 0.704) < 0.006, rho_ma
    lo, hi = rho_mi + 0.1 * (rho_ma - rho_mi), rho_ma - 0.1 * (rho_ma - rho_mi)
    zc = np.arange(nz, dtype=float)
    up = np.interp(hi, ra[70:50:-1], zc[70:50:-1])
    dn = np.interp(lo, ra[70:50:-1], zc[70:50:-1])
    assert 2.5 < dn - up < 7.0, dn - up


def _run_film(f0, rho_h, total):
    nz = 64
    o = Oracle(_params(1, 1, nz, g=3.6, psi=PSI_EXP, wall_z=True))
    o.init_from_populations(f0)
    ra, rb = o.density()
    rho_ma, rho_mi, rho_t = ra[5, 0, 0], ra[nz - 5, 0, 0], ra[nz - 5, 0, 0] + rb[nz - 5, 0, 0]
    o.set_sink(SINK_ZMAX, rho_h, 0.0)
    ts, xs = [], []
    for k in range(40):
        o.step(total // 40)
        ts.append((k + 1) * (total // 40))
        xs.append(o.diagnostics()["z_interface"])
    return np.array(ts), np.array(xs), rho_ma, rho_mi, rho_t


def test_film_interface_follows_sqrt_t_law(equilibrated_film64):
    """Eq. (xt), sign-fixed: (x_H - d0 - x_I)^2 grows linearly in t with slope
    2K, K = D (rho_mi - rho_H)/(rho_ma - rho_mi/2 - rho_H/2), D at the mean
    vapour composition. Only the quasi-static part (t > T/4) is fitted."""
    T = 100000
    slopes = {}
    for rho_h in (0.02, 0.03):
        ts, xs, rho_ma, rho_mi, rho_t = _run_film(equilibrated_film64, rho_h, T)
        assert np.all(np.diff(xs) < 0)  # rho_H < rho_mi: the film evaporates
        y = (63 - xs) ** 2
        sel = ts > T / 4
        p, res, *_ = np.polyfit(ts[sel], y[sel], 1, full=True)
        r2 = 1 - res[0] / np.sum((y[sel] - y[sel].mean()) ** 2)
        assert r2 > 0.999, r2
        ram = 0.5 * (rho_mi + rho_h)
        D = an.diffusion_small_gradient(ram, rho_t - ram, 3.6, "exp")
        K = an.film_rate_constant(D, rho_ma, rho_mi, rho_h)
        assert abs(p[0] / (2 * K) - 1) < 0.10, (rho_h, p[0], 2 * K)
        slopes[rho_h] = (p[0], K)
    # the evaporation rate scales with rho_mi - rho_H (Sec. III B)
    ratio_meas = slopes[0.02][0] / slopes[0.03][0]
    ratio_law = slopes[0.02][1] / slopes[0.03][1]
    assert abs(ratio_meas / ratio_law - 1) < 0.05, (ratio_meas, ratio_law)


def test_condensation_when_rho_h_above_minority(equilibrated_film64):
    """Sec. II C: rho_H above the minority density makes the film grow."""
    ts, xs, *_ = _run_film(equilibrated_film64, 0.05, 8000)
    assert xs[-1] > xs[0] + 0.05


# ---------------------------------------------------------------------------
# Droplet closed forms (Sec. III C): transcription checks of the readings.
# ---------------------------------------------------------------------------

def test_droplet_mass_derivative_matches_mass_integral():
    """Eq. (mass-df2) is d/dR of Eq. (drop-mass-1)."""
    RH, d0, rma, rmi, rh = 60.0, 2.5, 0.712, 0.037, 0.02
    for R in (12.0, 25.0, 40.0):
        h = 1e-3
        fd = (an.droplet_mass(R + h, RH, d0, rma, rmi, rh) - an.droplet_mass(R - h, RH, d0, rma, rmi, rh)) / (2 * h)
        assert abs(fd / an.droplet_dMdR(R, RH, d0, rma, rmi, rh) - 1) < 1e-4


def test_laplace_mass_derivative_is_total_derivative():
    """Eq. (drop-mass-df4) with d read as d0 is the total d/dR of Eq.
    (drop-mass-1) after substituting Eqs. (rho_ma) and (rho_mi)."""
    RH, d0, R0, gamma, rma0, rmi0, rh = 60.0, 2.5, 40.0, 0.01, 0.712, 0.037, 0.02

    def mass(R):
        rma, rmi = an.laplace_densities(R, R0, gamma, rma0, rmi0)
        return an.droplet_mass(R, RH, d0, rma, rmi, rh)

    for R in (10.0, 20.0, 35.0):
        h = 1e-3
        fd = (mass(R + h) - mass(R - h)) / (2 * h)
        assert abs(fd / an.droplet_dMdR_laplace(R, RH, d0, R0, gamma, rma0, rmi0, rh) - 1) < 1e-4


def test_rk4_reproduces_film_closed_form():
    """RK4 on the sign-fixed Eq. (xit) reproduces Eq. (xt)."""
    K, xh, d0, x0 = 3e-3, 127.0, 2.5, 64.0
    ts, ys = an.rk4(lambda x: -K / (xh - x - d0), x0, 2e5, 500.0)
    for t, y in zip(ts[::50], ys[::50]):
        assert abs(y - an.film_interface(t, x0, xh, d0, K)) < 1e-8


# ---------------------------------------------------------------------------
# Droplet radius laws (Sec. III C) on the oracle: surface tension from the
# Laplace law, then an evaporating droplet against RK4 of the sign-fixed
# Eqs. (mass-dfsum-sim) and (drop-r-df4).
# ---------------------------------------------------------------------------

CS2 = 1.0 / 3.0


def _bulk_pressure(ra, rb, g=3.6):
    """P = c_s^2 (rhoA + rhoB) + c_s^2 g psiA psiB, psi = 1 - exp(-rho): the
    continuum limit of the force of Eq. (sc) (the pressure of Sec. III C)."""
    return CS2 * (ra + rb) + CS2 * g * (1 - np.exp(-ra)) * (1 - np.exp(-rb))


@pytest.fixture(scope="module")
def oracle_surface_tension():
    """gamma from static cylinders (48 x 48 x 1: translation invariant along
    z) of the paper's fluid: P_in - P_out = gamma / R. The slowest
    composition mode of the box decays in ~500 steps, so 6000 steps settle
    the Laplace-shifted coexistence. R is the equimolar radius from the
    excess of A over the measured outside bulk."""
    n = 48
    c = (n - 1) / 2
    yy, xx = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    r = np.sqrt(xx ** 2 + yy ** 2)
    inv_r, dp = [], []
    for R0 in (8.0, 11.0, 14.0):
        a, b = li.droplet(n, n, 1, R0, center=(c, c, 0.0))
        o = Oracle(_params(n, n, 1, g=3.6, psi=PSI_EXP))
        o.init_from_density(a, b)
        o.step(6000)
        ra, rb = (x[0] for x in o.density())
        P = _bulk_pressure(ra, rb)
        inside, outside = r < R0 / 2, r > n / 2 - 3
        a_in, a_out = ra[inside].mean(), ra[outside].mean()
        R = math.sqrt((ra - a_out).sum() / (a_in - a_out) / math.pi)
        inv_r.append(1 / R)
        dp.append(P[inside].mean() - P[outside].mean())
    slope, icpt = np.polyfit(inv_r, dp, 1)
    return slope, icpt, inv_r, dp


@pytest.mark.slow
def test_laplace_law_of_cylinders(oracle_surface_tension):
    """Sec. III C's Laplace pressure: Delta P is linear in the curvature 1/R
    through the origin (measured gamma 0.0457, intercept 4 % of Delta P)."""
    gamma, icpt, inv_r, dp = oracle_surface_tension
    assert gamma > 0
    fit = np.polyval([gamma, icpt], inv_r)
    assert np.max(np.abs(fit - dp)) < 0.02 * max(dp)
    assert abs(icpt) < 0.05 * max(dp), icpt / max(dp)


def _wave_diffusion_oracle(ma, mb, nz=64, amp=1e-4, every=200):
    """Decay rate of a composition wave exp(-D k^2 t) (Eq. (fick2)) on the
    oracle at mean composition (ma, mb), paper fluid."""
    o = Oracle(_params(1, 1, nz, g=3.6, psi=PSI_EXP))
    a, b = li.sinus(1, 1, nz, ma, mb, amp)
    o.init_from_density(a, b)
    s = np.sin(2 * np.pi * np.arange(nz) / nz)
    amps, ts = [], []
    for k in range(9):
        if k:
            o.step(every)
        amps.append((o.density()[0][:, 0, 0] - ma) @ s / (s @ s))
        ts.append(every * k)
    return -np.polyfit(ts[2:], np.log(amps[2:]), 1)[0] / (2 * np.pi / nz) ** 2


@pytest.mark.slow
def test_droplet_shrinks_like_the_radius_laws(oracle_surface_tension):
    """Sec. III C on the oracle: a droplet of the paper's fluid (R0 = 14 in
    48^3, spherical sink R_H = N/2 - 1 = 23, rho_H = 0.02), equilibrated
    2000 steps, then evaporating until R < 9.5.

    D enters both laws as a factor. The small-gradient formula of Eq.
    (diffu-t-1) assumes grad rho^B = -grad rho^A, which does not hold at the
    vapour's asymmetric composition, so D is measured on the oracle from a
    composition wave at the mean vapour composition (0.84 of the formula).
    With it, R(t) follows both laws to within half a lattice unit while the
    diameter exceeds 20 (the range the paper fits; measured 0.25 and 0.30).

    The paper's claim that the Laplace-corrected law is the better one at
    small radii is checked on the shape of R(t), which does not depend on D:
    the ratio of the shrink rates at R = 10 and R = 13. Measured 1.075, plain
    law 0.966, Laplace law 0.977: the droplet speeds up as it shrinks, which
    only the Laplace term (the minority density rising with the Laplace
    pressure) produces, and the Laplace law is the closer one."""
    gamma = oracle_surface_tension[0]
    n, R0, RH, rho_h, d0 = 48, 14.0, 23.0, 0.02, 2.5
    o = Oracle(_params(n, n, n, g=3.6, psi=PSI_EXP, sink=SINK_NONE, rho_h=rho_h, sink_radius=RH,
                       phi_delta=(0.675, -0.675)))
    a, b = li.droplet(n, n, n, R0)
    o.init_from_density(a, b)
    o.step(2000)
    ra, rb = o.density()
    c = n // 2
    rho_ma0 = ra[c - 2:c + 2, c - 2:c + 2, c - 2:c + 2].mean()
    zz, yy, xx = np.meshgrid(*(np.arange(n) - (n - 1) / 2,) * 3, indexing="ij")
    r = np.sqrt(xx ** 2 + yy ** 2 + zz ** 2)
    shell = (r > RH - 4) & (r < RH - 1)
    rho_mi0, rho_t = ra[shell].mean(), (ra + rb)[shell].mean()
    o.set_sink(SINK_SPHERE, rho_h, RH)
    ts, rs = [0.0], [o.diagnostics()["r_droplet"]]
    while rs[-1] > 9.5:
        o.step(250)
        ts.append(ts[-1] + 250)
        rs.append(o.diagnostics()["r_droplet"])
        assert ts[-1] < 12000, "droplet must evaporate"
    ts, rs = np.array(ts), np.array(rs)
    assert np.all(np.diff(rs) < 0)
    ram = 0.5 * (rho_mi0 + rho_h)
    D = _wave_diffusion_oracle(ram, rho_t - ram)
    assert 0.7 < D / an.diffusion_small_gradient(ram, rho_t - ram, 3.6, "exp") < 1.0

    def plain(R):
        return an.droplet_rate_plain(R, RH, d0, D, rho_ma0, rho_mi0, rho_h)

    def laplace(R):
        return an.droplet_rate_laplace(R, RH, d0, D, rs[0], gamma, rho_ma0, rho_mi0, rho_h)

    big = rs > 10.0
    for law in (plain, laplace):
        t_law, r_law = an.rk4(law, rs[0], ts[-1], 25.0)
        err = np.max(np.abs(rs - np.interp(ts, t_law, r_law))[big])
        assert err < 0.5, (law.__name__, err)
    rate = -np.gradient(rs, ts)

    def measured(R):
        return np.interp(-R, -rs, rate)

    m = measured(10.0) / measured(13.0)
    p = plain(10.0) / plain(13.0)
    q = laplace(10.0) / laplace(13.0)
    print(f"rate(10)/rate(13): measured {m:.4f}, plain law {p:.4f}, Laplace law {q:.4f}")
    assert q > p                         # the Laplace term speeds small droplets up
    assert abs(m - q) <= abs(m - p)      # and the Laplace law is the closer one
