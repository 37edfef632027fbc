"""GPU parity of the single-component multiphase form (the method carried over
to the multiphase pseudopotential model, Sec. I): one component whose force
of Eq. (sc) takes itself as the partner, the evaporation boundary holding it
at rho_H and booking what it removes (Sec. II C).

Bars: FP64 populations within 1e-12 of max|f|; FP32S within 2e-6 of max|f|
(one rounding of the stored deviations per step); masses and E within 1e-13
(FP64) and 1e-6 (FP32S) of the total mass.
"""
import numpy as np
import pytest
import torch

import lbinputs as li
from oracle import analytic as an
from oracle.oracle import PSI_EXP, PSI_RHO, SINK_FACES, SINK_NONE, SINK_SPHERE, SINK_ZMAX, Oracle, OracleParams

pytestmark = pytest.mark.gpu

SINK_CODE = {"none": SINK_NONE, "zmax": SINK_ZMAX, "faces": SINK_FACES, "sphere": SINK_SPHERE}


@pytest.fixture(scope="module")
def lb():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1701_03637_amd as lb
    lb.load_library()
    return lb


CASES = [
    # lattice, psi, g, sink, wall_z, solid planes, tau
    ((13, 7, 9), "exp", -4.5, "none", False, 0, 1.0),
    ((13, 7, 11), "exp", -5.0, "zmax", True, 0, 1.0),
    ((9, 10, 11), "rho", -1.2, "faces", False, 0, 0.8),
    ((11, 11, 11), "exp", -4.5, "sphere", False, 0, 1.3),
    ((12, 6, 14), "exp", -5.0, "zmax", False, 2, 1.0),
    ((70, 3, 5), "exp", -4.5, "faces", False, 0, 1.0),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision,tol,tol_m", [("fp64", 1e-12, 1e-13), ("fp32s", 2e-6, 1e-6)])
def test_single_component_matches_oracle(lb, case, precision, tol, tol_m):
    (nx, ny, nz), psi, g, sink, wall_z, h, tau = case
    rng = np.random.default_rng(3)
    p = lb.make_params(nx, ny, nz, g=g, psi=psi, tau=(tau, 1.0), precision=precision, sink=sink, rho_h=0.12,
                       sink_radius=0.4 * nz, wall_z=wall_z, solid_z=h, wall_rho=(0.9, 0.0), ncomp=1,
                       shift=(0.3, 0.0), phi_delta=(1.9, 0.16))
    sim = lb.Sim(p)
    orc = Oracle(OracleParams(nx, ny, nz, g=g, psi=PSI_EXP if psi == "exp" else PSI_RHO, tau=(tau, 1.0),
                              sink=SINK_CODE[sink], rho_h=0.12, sink_radius=0.4 * nz, wall_z=wall_z, solid_z=h,
                              wall_rho=(0.9, 0.0), ncomp=1, phi_delta=(1.9, 0.16)))
    f0 = li.random_populations(nx, ny, nz, seed=int(rng.integers(1 << 30)), base_a=0.3, base_b=0.0, amp=0.05)
    sim.init_from_populations(f0[:1])
    orc.init_from_populations(f0)
    sim.step(7)
    orc.step(7)
    got = sim.populations().cpu().numpy()
    ref = orc.populations()[:1]
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)), np.max(np.abs(got - ref))
    dg, do = sim.diagnostics(), orc.diagnostics()
    tot = do["mass"][0]
    assert abs(dg["mass"][0] - do["mass"][0]) <= tol_m * tot
    assert dg["mass"][1] == 0.0
    assert abs(dg["evaporated"] - do["evaporated"]) <= tol_m * tot
    assert np.allclose(dg["momentum"], do["momentum"], atol=10 * tol_m * tot, rtol=0)
    ra, rb, u = sim.observables()
    assert not torch.any(rb)
    assert np.max(np.abs(ra.cpu().numpy() - orc.density()[0])) <= 19 * tol * np.max(np.abs(ref))
    if precision == "fp64":
        assert np.max(np.abs(u.cpu().numpy() - orc.velocity())) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
def test_single_component_schedules_bitwise(lb, precision):
    """Every tile schedule gives the same bits (ragged tiles, odd chunks)."""
    nx, ny, nz = 70, 23, 19
    f0 = li.random_populations(nx, ny, nz, seed=9, base_a=0.3, base_b=0.0, amp=0.05)[:1]

    def run(t):
        sim = lb.Sim(lb.make_params(nx, ny, nz, psi="exp", g=-4.5, sink="faces", rho_h=0.12, precision=precision,
                                    ncomp=1, shift=(0.3, 0.0)))
        sim.set_tiles(*t)
        sim.init_from_populations(f0)
        sim.step(7)
        return sim.populations()
    ref = run((256, 0, 0, 0, 1))
    for t in ((512, 0, 0, 0, 1), (256, 16, 4, 3, 1), (512, 32, 8, 7, 0), (256, 64, 2, 5, 1)):
        assert torch.equal(run(t), ref), t


@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
def test_single_component_coexistence_and_evaporation(lb, precision):
    """A liquid slab of the multiphase fluid (g = -5) in its vapour settles at
    the equal-area coexistence densities (vapour within 1 %, liquid within
    0.1 %, as the oracle does), with its mass conserved; then the top plane
    is held below the vapour density and the film evaporates, M + E = M(0)
    to the storage's bar."""
    G, nz = -5.0, 128
    rv, rl = an.coexistence_single(G)
    p = lb.make_params(4, 4, nz, g=G, psi="exp", precision=precision, ncomp=1, shift=(rv, 0.0),
                       phi_delta=(rl, rv), rho_h=0.5 * rv, solid_z=2, wall_rho=(rl, 0.0))
    sim = lb.Sim(p)
    sim.set_graph(100)
    z = np.arange(nz)
    sim.init_from_density(np.broadcast_to(np.where((z >= 2) & (z < 64), rl, rv).reshape(nz, 1, 1),
                                          (nz, 4, 4)).copy())
    m0 = sim.diagnostics()["mass"][0]
    sim.step(20000)
    r = sim.density(0).cpu().numpy()[:, 0, 0]
    print(f"{precision}: vapour {r[90:110].mean():.5f} (rule {rv:.5f}), liquid {r[20:44].mean():.5f} (rule {rl:.5f})")
    assert abs(r[90:110].mean() / rv - 1) < 0.01
    assert abs(r[20:44].mean() / rl - 1) < 0.001
    d0 = sim.diagnostics()
    bar = 2e-12 if precision == "fp64" else 1e-6   # FP64: 1e-13 per 10^3 steps
    assert abs(d0["mass"][0] - m0) <= bar * m0
    sim.set_sink("zmax", 0.5 * rv)
    sim.step(5000)
    d1 = sim.diagnostics()
    print(f"{precision}: z_I {d0['z_interface']:.3f} -> {d1['z_interface']:.3f}, E = {d1['evaporated']:.4f}")
    assert d1["evaporated"] > 0 and d1["z_interface"] < d0["z_interface"]
    assert abs(d1["mass"][0] + d1["evaporated"] - d0["mass"][0]) <= bar * d0["mass"][0]
