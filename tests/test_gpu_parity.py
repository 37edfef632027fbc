"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances:
  FP64  - populations within 1e-12 of max|f| (rounding order only);
  FP32S - densities within 1e-5, populations within 2e-6 of max|f|;
  FP16S - densities within 1e-3.
They are derived from the storage unit roundoff (2^-24, 2^-11 of the stored
deviation) accumulated over the steps of each case; see the design notes.
"""
import math

import numpy as np
import pytest
import torch

import lbinputs as li
from oracle.oracle import (PSI_EXP, PSI_RHO, SINK_FACES, SINK_NONE, SINK_SPHERE, SINK_ZMAX, Oracle,
                           OracleParams)

pytestmark = pytest.mark.gpu

SINK_CODE = {"none": SINK_NONE, "zmax": SINK_ZMAX, "faces": SINK_FACES, "sphere": SINK_SPHERE}


@pytest.fixture(scope="module")
def lb():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1701_03637_amd as lb
    lb.load_library()
    return lb


def _pair(lb, nx, ny, nz, *, precision="fp64", psi="rho", g=0.9, tau=(1.0, 1.0), wall_z=False, sink="none",
          rho_h=0.04, sink_radius=0.0, shift=(0.04, 0.70), phi_delta=(0.66, -0.66)):
    p = lb.make_params(nx, ny, nz, wall_z=wall_z, tau=tau, g=g, psi=psi, precision=precision, shift=shift,
                       sink=sink, rho_h=rho_h, sink_radius=sink_radius, phi_delta=phi_delta)
    sim = lb.Sim(p)
    orc = Oracle(OracleParams(nx, ny, nz, wall_z=wall_z, tau=tau, g=g, psi=PSI_EXP if psi == "exp" else PSI_RHO,
                              sink=SINK_CODE[sink], rho_h=rho_h, sink_radius=sink_radius, phi_delta=phi_delta))
    return sim, orc


def _cmp_pops(sim, orc, tol_rel):
    got = sim.populations().cpu().numpy()
    ref = orc.populations()
    err = np.max(np.abs(got - ref))
    scale = np.max(np.abs(ref))
    assert err <= tol_rel * scale, f"max |df| = {err:.3e} (scale {scale:.3e})"
    return err


@pytest.mark.parametrize("case", [
    dict(dims=(13, 7, 9), psi="exp", g=2.2, sink="none", wall_z=False, steps=6),
    dict(dims=(13, 7, 9), psi="rho", g=0.9, sink="zmax", wall_z=True, steps=6),
    dict(dims=(9, 10, 11), psi="exp", g=1.5, sink="faces", wall_z=False, steps=5),
    dict(dims=(11, 11, 11), psi="rho", g=0.9, sink="sphere", wall_z=False, steps=5, sink_radius=4.2,
         tau=(0.8, 1.3)),
    dict(dims=(1, 1, 16), psi="exp", g=3.6, sink="zmax", wall_z=True, steps=8),
    dict(dims=(70, 3, 5), psi="rho", g=1.1, sink="faces", wall_z=False, steps=4),
])
def test_fp64_random_populations_match_oracle(lb, case):
    nx, ny, nz = case["dims"]
    sim, orc = _pair(lb, nx, ny, nz, psi=case["psi"], g=case["g"], sink=case["sink"], wall_z=case["wall_z"],
                     rho_h=0.03, sink_radius=case.get("sink_radius", 0.0), tau=case.get("tau", (1.0, 1.0)))
    f0 = li.random_populations(nx, ny, nz, seed=7, base_a=0.3, base_b=0.4, amp=0.05)
    sim.init_from_populations(f0)
    orc.init_from_populations(f0)
    _cmp_pops(sim, orc, 1e-14)   # initial sink reset
    for _ in range(case["steps"]):
        sim.step(1)
        orc.step(1)
    _cmp_pops(sim, orc, 1e-12)
    dg, do = sim.diagnostics(), orc.diagnostics()
    tot = do["mass"][0] + do["mass"][1]
    for c in range(2):
        assert abs(dg["mass"][c] - do["mass"][c]) <= 1e-13 * tot
    assert abs(dg["evaporated"] - do["evaporated"]) <= 1e-13 * tot
    assert abs(dg["evap_rate"] - do["evap_rate"]) <= 1e-13 * tot
    assert np.allclose(dg["momentum"], do["momentum"], atol=1e-12 * tot, rtol=0)


@pytest.mark.parametrize("dims,sink,wall_z,radius", [
    ((4096, 2, 3), "none", False, 0.0),
    ((3, 4096, 2), "sphere", False, 1000.0),
    ((2, 3, 4096), "zmax", True, 0.0),
    ((1, 1, 4096), "zmax", True, 0.0),
])
def test_fp64_size_limits_match_oracle(lb, dims, sink, wall_z, radius):
    """Lattices of the largest extent (4096) along one axis and one to three
    nodes along the others, in the default schedule: a long x or y split
    into many tiles, thousands of short z chunks, stencils that wrap inside
    one- and two-node extents, and a sphere whose sink splits the long axis."""
    nx, ny, nz = dims
    sim, orc = _pair(lb, nx, ny, nz, psi="exp", g=2.0, sink=sink, wall_z=wall_z, rho_h=0.03, sink_radius=radius)
    f0 = li.random_populations(nx, ny, nz, seed=11, base_a=0.3, base_b=0.4, amp=0.05)
    sim.init_from_populations(f0)
    orc.init_from_populations(f0)
    sim.step(4)
    orc.step(4)
    _cmp_pops(sim, orc, 1e-12)
    dg, do = sim.diagnostics(), orc.diagnostics()
    tot = do["mass"][0] + do["mass"][1]
    for c in range(2):
        assert abs(dg["mass"][c] - do["mass"][c]) <= 1e-13 * tot
    assert abs(dg["evaporated"] - do["evaporated"]) <= 1e-13 * tot


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32s", 2e-6)])
@pytest.mark.parametrize("dims,wall_z,sink", [((1, 1, 1), False, "none"), ((1, 1, 1), True, "none"),
                                              ((1, 1, 2), True, "zmax"), ((2, 1, 1), False, "none")])
def test_smallest_lattices_match_oracle(lb, precision, tol, dims, wall_z, sink):
    """Degenerate lattices: every neighbour of a 1x1x1 node is the node itself
    (periodic), or, walled, both z directions reflect off the same plane; a
    walled 1x1x2 column whose top plane is the sink."""
    nx, ny, nz = dims
    sim, orc = _pair(lb, nx, ny, nz, precision=precision, psi="exp", g=2.0, sink=sink, wall_z=wall_z, rho_h=0.03)
    f0 = li.random_populations(nx, ny, nz, seed=13, base_a=0.3, base_b=0.4, amp=0.05)
    sim.init_from_populations(f0)
    orc.init_from_populations(f0)
    sim.step(6)
    orc.step(6)
    _cmp_pops(sim, orc, tol)
    dg, do = sim.diagnostics(), orc.diagnostics()
    tot = do["mass"][0] + do["mass"][1]
    assert abs(dg["mass"][0] + dg["mass"][1] - tot) <= 10 * tol * tot


def test_zero_and_negative_step_counts(lb):
    """step(0) launches nothing and leaves state and step counter as they
    are; a negative count is an argument error that changes nothing."""
    nx, ny, nz = 12, 10, 8
    sim = lb.Sim(lb.make_params(nx, ny, nz, psi="exp", g=2.0, sink="faces", rho_h=0.03, precision="fp32s"))
    sim.init_from_populations(li.random_populations(nx, ny, nz, seed=2, base_a=0.3, base_b=0.4, amp=0.05))
    sim.step(3)
    before = sim.populations().clone()
    sim.step(0)
    assert torch.equal(sim.populations(), before)
    assert sim.diagnostics()["step"] == 3
    with pytest.raises(lb.LbscError, match="negative"):
        sim.step(-1)
    assert torch.equal(sim.populations(), before)
    assert sim.diagnostics()["step"] == 3


def test_fp64_film_config_full_run(lb):
    """4x4x128 film, psi = rho, g = 0.9, sink on z = 127, wall, 1000 steps."""
    w = li.film_small()
    sim, orc = _pair(lb, w.nx, w.ny, w.nz, psi=w.psi, g=w.g, sink=w.sink, wall_z=w.wall_z, rho_h=w.rho_h)
    a, b = w.densities()
    sim.init_from_density(a, b)
    orc.init_from_density(a, b)
    for chunk in (1, 99, 400, 500):
        sim.step(chunk)
        orc.step(chunk)
        _cmp_pops(sim, orc, 1e-12)
    dg, do = sim.diagnostics(), orc.diagnostics()
    assert dg["step"] == do["step"] == 1000
    tot = do["mass"][0] + do["mass"][1]
    assert abs(dg["mass"][0] - do["mass"][0]) <= 1e-13 * tot
    assert abs(dg["evaporated"] - do["evaporated"]) <= 1e-13 * tot
    assert abs(dg["z_interface"] - do["z_interface"]) <= 1e-9
    ra, rb, u = sim.observables()
    ora, orb = orc.density()
    ou = orc.velocity()
    assert np.max(np.abs(ra.cpu().numpy() - ora)) < 1e-13
    assert np.max(np.abs(u.cpu().numpy() - ou)) < 1e-13


def test_fp64_droplet_ragged_tiles_and_sink_switch(lb):
    """Droplet in 37x29x33 (ragged tiles), equilibrated without sink, then the
    sink is switched on mid-run (Sec. III C workflow)."""
    nx, ny, nz = 37, 29, 33
    sim, orc = _pair(lb, nx, ny, nz, psi="exp", g=3.6, sink="none", rho_h=0.02, phi_delta=(0.675, -0.675))
    a, b = li.droplet(nx, ny, nz, 8.0)
    sim.init_from_density(a, b)
    orc.init_from_density(a, b)
    sim.step(30)
    orc.step(30)
    _cmp_pops(sim, orc, 1e-12)
    sim.set_sink("sphere", 0.02, 13.5)
    orc.set_sink(SINK_SPHERE, 0.02, 13.5)
    d_s, d_o = sim.diagnostics(), orc.diagnostics()
    assert abs(d_s["evaporated"] - d_o["evaporated"]) < 1e-12
    sim.step(40)
    orc.step(40)
    _cmp_pops(sim, orc, 1e-12)
    d_s, d_o = sim.diagnostics(), orc.diagnostics()
    assert abs(d_s["evaporated"] - d_o["evaporated"]) <= 1e-12 * d_o["mass"][0]
    assert abs(d_s["r_droplet"] - d_o["r_droplet"]) <= 1e-10
    sim.set_sink("none", 0.02, 0.0)
    orc.set_sink(SINK_NONE, 0.02, 0.0)
    sim.step(5)
    orc.step(5)
    _cmp_pops(sim, orc, 1e-12)


@pytest.mark.parametrize("tiles", [(256, 0, 0, 0, 1), (512, 0, 0, 0, 1), (256, 16, 4, 3, 1), (512, 32, 8, 7, 1),
                                   (256, 64, 2, 5, 1), (256, 0, 0, 0, 2), (512, 32, 8, 7, 2), (256, 64, 2, 5, 2),
                                   (256, 70, 3, 4, 1), (512, 256, 2, 6, 2)])
@pytest.mark.parametrize("precision", ["fp64", "fp32s", "fp16s", "fp16n"])
def test_tile_schedules_bitwise_identical(lb, tiles, precision):
    """The result does not depend on the tile schedule (catches LDS halo races,
    ragged-tile indexing, and inlined copies of a store that round
    differently: odd z chunks store a plane through the other copy)."""
    nx, ny, nz = 70, 23, 19
    f0 = li.random_populations(nx, ny, nz, seed=3, base_a=0.3, base_b=0.4, amp=0.05)
    ref = lb.Sim(lb.make_params(nx, ny, nz, psi="exp", g=2.0, sink="faces", rho_h=0.03, precision=precision))
    ref.init_from_populations(f0)
    ref.step(7)
    sim = lb.Sim(lb.make_params(nx, ny, nz, psi="exp", g=2.0, sink="faces", rho_h=0.03, precision=precision))
    sim.set_tiles(*tiles)
    sim.init_from_populations(f0)
    sim.step(7)
    assert torch.equal(sim.populations(), ref.populations())


PIPE_CASES = [
    # (lattice, wall_z, sink, tiles): ragged tiles, tiles spanning the whole
    # x and/or y extent (halo wraps inside the tile), z chunks of 1 and 2
    ((70, 23, 19), False, "faces", (256, 64, 2, 5, 3)),
    ((70, 23, 19), False, "faces", (256, 16, 4, 3, 3)),
    ((70, 23, 19), False, "faces", (512, 32, 8, 7, 3)),
    ((64, 23, 19), False, "faces", (256, 64, 4, 5, 3)),
    ((20, 12, 19), False, "faces", (256, 20, 12, 4, 3)),
    ((20, 12, 19), False, "faces", (256, 16, 12, 4, 3)),
    ((16, 8, 40), True, "zmax", (256, 8, 8, 6, 3)),
    ((16, 8, 40), True, "zmax", (256, 16, 8, 1, 3)),
    ((40, 24, 21), False, "faces", (256, 32, 8, 2, 3)),
    ((128, 6, 9), False, "faces", (256, 128, 2, 0, 0)),
    ((150, 7, 9), False, "faces", (512, 150, 3, 4, 3)),
    ((150, 7, 9), False, "faces", (512, 0, 0, 0, 3)),
    ((200, 5, 11), True, "zmax", (512, 200, 2, 0, 3)),
    ((40, 24, 21), False, "sphere", (256, 40, 6, 4, 3), (0.8, 1.3)),
    # extents at the 4096 limit, default tiles and chunks
    ((4096, 2, 3), False, "none", (256, 0, 0, 0, 3)),
    ((2, 3, 4096), True, "zmax", (512, 0, 0, 0, 3)),
]


@pytest.mark.parametrize("case", PIPE_CASES)
@pytest.mark.parametrize("precision", ["fp32s", "fp16s", "fp64", "fp16n"])
def test_pipelined_variant_bitwise_identical(lb, case, precision):
    """The pipelined step (one plane of loads ahead, four psi slots, halo
    wrapped inside tiles that span x or y, chunks marching up and down; FP16N
    with its rest values through an LDS ring) gives the same bits as the
    register-keeping step, and books the same evaporated mass; one case has
    tau^A != tau^B and a spherical sink."""
    (nx, ny, nz), wall, sink, tiles = case[:4]
    tau = case[4] if len(case) > 4 else (1.0, 1.0)
    if precision == "fp64" and tiles[0] != 256:
        pytest.skip("the FP64 pipelined step runs 256-thread blocks")
    if precision == "fp16n" and tiles[1] > 0 and (tiles[1] + 4) * (tiles[2] + 4) > 3 * tiles[0]:
        pytest.skip("the FP16N rest footprint (tw + 4)(th + 4) exceeds 3 nt")
    f0 = li.random_populations(nx, ny, nz, seed=5, base_a=0.3, base_b=0.4, amp=0.05)

    def run(t):
        sim = lb.Sim(lb.make_params(nx, ny, nz, wall_z=wall, psi="exp", g=2.0, sink=sink, rho_h=0.03,
                                    sink_radius=0.4 * nz, tau=tau, precision=precision))
        sim.set_tiles(*t)
        sim.init_from_populations(f0)
        sim.step(7)
        return sim
    ref, sim = run((256, 0, 0, 0, 1)), run(tiles if precision != "fp64" or tiles[4] != 0 else (256, *tiles[1:4], 3))
    assert sim.tiles()[4] == 3
    assert torch.equal(sim.populations(), ref.populations())
    e_ref, e = ref.diagnostics()["evaporated"], sim.diagnostics()["evaporated"]
    assert abs(e - e_ref) <= 1e-12 * max(1.0, abs(e_ref))


def test_batched_instances_equal_separate_runs(lb):
    shapes = [(24, 24, 24, 0.85, 0.03), (40, 40, 40, 0.97, 0.05), (17, 21, 13, 0.9, 0.02)]
    params = [lb.make_params(n0, n1, n2, g=g, sink="faces", rho_h=rh, precision="fp32s")
              for n0, n1, n2, g, rh in shapes]
    batch = lb.Sim(params)
    singles = []
    for k, (n0, n1, n2, g, rh) in enumerate(shapes):
        a, b = li.droplet(n0, n1, n2, 0.2 * n0)
        batch.init_from_density(a, b, inst=k)
        s = lb.Sim(params[k])
        s.init_from_density(a, b)
        singles.append(s)
    batch.step(25)
    for k, s in enumerate(singles):
        s.step(25)
        assert torch.equal(batch.populations(inst=k), s.populations())
        db, ds = batch.diagnostics(inst=k), s.diagnostics()
        assert db["mass"] == ds["mass"] and db["evaporated"] == ds["evaporated"]


def test_graph_replay_and_checkpoint_bitwise(lb):
    nx, ny, nz = 32, 30, 28
    p = lb.make_params(nx, ny, nz, g=0.9, sink="faces", rho_h=0.03, precision="fp32s")
    a, b = li.droplet(nx, ny, nz, 7.0)
    ref = lb.Sim(p)
    ref.init_from_density(a, b)
    ref.step(41)
    g = lb.Sim(p)
    g.set_graph(8)
    g.init_from_density(a, b)
    g.step(17)
    blob = g.checkpoint()
    g.step(24)
    assert torch.equal(g.populations(), ref.populations())
    r = lb.Sim(p)
    r.init_from_density(a, a)  # different state, overwritten by the restore
    r.restore(blob)
    r.step(24)
    assert torch.equal(r.populations(), ref.populations())
    dr, dref = r.diagnostics(), ref.diagnostics()
    assert dr["step"] == dref["step"] == 41
    assert abs(dr["evaporated"] - dref["evaporated"]) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32s", "fp16n"])
def test_every_graph_replay_matches_eager_steps(lb, precision):
    """Each replay of the step graph gives the bits of the same steps launched
    one by one. Eager work (diagnostics, with their synchronisation, and one
    eager step that flips the buffer parity) runs between the replays, so both
    of the context's graphs (one per parity) are replayed several times."""
    nx, ny, nz = 24, 20, 26
    p = lb.make_params(nx, ny, nz, g=3.6, psi="exp", sink="sphere", rho_h=0.02, sink_radius=9.5,
                       precision=precision)
    a, b = li.droplet(nx, ny, nz, 6.0)
    ref = lb.Sim(p)
    ref.init_from_density(a, b)
    g = lb.Sim(p)
    g.set_graph(4)
    g.init_from_density(a, b)
    g.step(1)                # the first step after an initialisation is never replayed
    ref.step(1)
    for k in range(6):
        g.step(4)            # one replay
        ref.step(4)
        assert torch.equal(g.populations(), ref.populations()), f"replay {k}"
        dg, dr = g.diagnostics(), ref.diagnostics()
        assert dg["step"] == dr["step"]
        assert dg["evaporated"] == dr["evaporated"], f"replay {k}"
        if k % 2 == 0:
            g.step(1)        # eager: the next replay uses the other parity's graph
            ref.step(1)


@pytest.mark.parametrize("precision,tol_rho", [("fp32s", 1e-5), ("fp16n", 2e-4),
                                               pytest.param("fp16s", 1e-3, marks=pytest.mark.xfail(
                                                   reason="constant-shift FP16 quantises the slow dense-phase "
                                                          "dynamics of this sharp film; FP16N fixes it", strict=True))])
def test_reduced_precision_film_against_oracle(lb, precision, tol_rho):
    w = li.film_small()
    sim, orc = _pair(lb, w.nx, w.ny, w.nz, precision=precision, psi=w.psi, g=w.g, sink=w.sink, wall_z=w.wall_z,
                     rho_h=w.rho_h)
    a, b = w.densities()
    sim.init_from_density(a, b)
    orc.init_from_density(a, b)
    sim.step(w.steps)
    orc.step(w.steps)
    ra = sim.density(0).cpu().numpy()
    ora, orb = orc.density()
    err = np.max(np.abs(ra - ora))
    print(f"{precision}: max |drho_A| = {err:.3e}")
    assert err < tol_rho, err
    dg, do = sim.diagnostics(), orc.diagnostics()
    tot = do["mass"][0] + do["mass"][1]
    drift = abs(dg["mass"][0] + dg["mass"][1] - tot) / tot
    print(f"{precision}: total-mass drift {drift:.3e}")
    assert drift < {"fp32s": 1e-6, "fp16n": 1e-6}.get(precision, 1e-3), drift
    assert abs(dg["z_interface"] - do["z_interface"]) < (0.01 if precision == "fp32s" else 0.1)


@pytest.mark.parametrize("precision,tol", [("fp32s", 2e-6), ("fp16s", 2e-3), ("fp16n", 2e-5)])
def test_reduced_precision_droplet_against_oracle(lb, precision, tol):
    nx = ny = nz = 40
    sim, orc = _pair(lb, nx, ny, nz, precision=precision, g=0.9, sink="faces", rho_h=0.04)
    a, b = li.droplet(nx, ny, nz, 8.0)
    sim.init_from_density(a, b)
    orc.init_from_density(a, b)
    sim.step(50)
    orc.step(50)
    got = sim.density(0).cpu().numpy()
    ref = orc.density()[0]
    print(f"{precision}: droplet max |drho_A| = {np.max(np.abs(got - ref)):.3e}")
    assert np.max(np.abs(got - ref)) < tol * 10
    dg, do = sim.diagnostics(), orc.diagnostics()
    tot = do["mass"][0] + do["mass"][1]
    assert abs(dg["mass"][0] + dg["evaporated"] - (do["mass"][0] + do["evaporated"])) / tot < tol


def test_tuner_leaves_a_schedule_with_identical_results(lb):
    """lbsc_tune times every candidate schedule on the live state (re-timing
    its three fastest) and keeps the best; what it keeps must be a valid
    schedule giving the same bits as the default one, and the graph setting
    must survive the tuning."""
    nx, ny, nz = 40, 36, 32
    p = lb.make_params(nx, ny, nz, psi="exp", g=2.0, sink="faces", rho_h=0.03, precision="fp32s")
    sim = lb.Sim(p)
    sim.set_graph(4)
    a, b = li.droplet(nx, ny, nz, 8.0)
    sim.init_from_density(a, b)
    chosen = sim.tune(3)
    assert sim.tiles() == chosen
    assert chosen[0] in (256, 512) and chosen[4] in (1, 2, 3)
    f = sim.populations()
    ref = lb.Sim(p)
    for s in (sim, ref):
        s.init_from_populations(f)
        s.step(6)
    assert torch.equal(sim.populations(), ref.populations())
    d = sim.diagnostics()
    assert d["nonfinite"] == 0
