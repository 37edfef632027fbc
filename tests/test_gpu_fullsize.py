"""Parity at the full workload sizes, in the launch configuration bench.py times.

128^3 droplet: the whole lattice against the oracle after a few steps.
512^3 droplet: sampled nodes against the oracle run on a window around each
sample (the state at a node after t steps depends only on nodes within 2t:
one hop for the pull, one for the force stencil), plus whole-lattice
properties (sink mass bookkeeping, mirror symmetry of the centred droplet).
"""
import numpy as np
import pytest
import torch

import lbinputs as li
from oracle.oracle import PSI_RHO, SINK_FACES, SINK_NONE, Oracle, OracleParams

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1701_03637_amd as lb
    lb.load_library()
    return lb


def _sim(lb, w, precision):
    return lb.Sim(lb.make_params(w.nx, w.ny, w.nz, wall_z=w.wall_z, g=w.g, psi=w.psi, precision=precision,
                                 sink=w.sink, rho_h=w.rho_h))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32s", 2e-6)])
def test_droplet128_whole_lattice(lb, precision, tol):
    w = li.droplet_128()
    steps = 3
    sim = _sim(lb, w, precision)
    a, b = w.densities()
    sim.init_from_density(a, b)
    sim.step(steps)
    got = sim.populations().cpu().numpy()
    orc = Oracle(OracleParams(w.nx, w.ny, w.nz, g=w.g, psi=PSI_RHO, sink=SINK_FACES, rho_h=w.rho_h))
    orc.init_from_density(a, b)
    orc.step(steps)
    ref = orc.populations()
    err = np.max(np.abs(got - ref))
    assert err < tol, err
    d, do = sim.diagnostics(), orc.diagnostics()
    assert abs(d["evaporated"] - do["evaporated"]) < tol * w.nodes


def _window_reference(a, b, center, half, steps, g):
    """Oracle on a periodic window of side 2*half+1 cut from the global field."""
    idx = [np.arange(c - half, c + half + 1) for c in center]  # z, y, x
    wa = a.take(idx[0], axis=0, mode="wrap").take(idx[1], axis=1, mode="wrap").take(idx[2], axis=2, mode="wrap")
    wb = b.take(idx[0], axis=0, mode="wrap").take(idx[1], axis=1, mode="wrap").take(idx[2], axis=2, mode="wrap")
    n = 2 * half + 1
    o = Oracle(OracleParams(n, n, n, g=g, psi=PSI_RHO, sink=SINK_NONE))
    o.init_from_density(wa, wb)
    o.step(steps)
    return o.populations()[:, :, half, half, half]


def test_droplet512_fp32s_sampled_and_properties(lb):
    w = li.droplet_512()
    steps = 3
    sim = _sim(lb, w, "fp32s")
    a, b = w.densities()
    sim.init_from_density(a, b)
    d0 = sim.diagnostics()
    sim.step(steps)
    f = sim.populations()  # (2, 19, nz, ny, nx) on the device, FP64
    rng = np.random.default_rng(5)
    # interior samples (no sink node within the dependency radius), half of
    # them on the droplet interface where gradients are largest
    samples = [tuple(int(v) for v in rng.integers(10, 502, 3)) for _ in range(8)]
    c = (w.nx - 1) / 2
    for k in range(8):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        p = np.rint(c + 120.0 * d).astype(int)
        samples.append((int(p[2]), int(p[1]), int(p[0])))
    half = 2 * steps + 2
    for (z, y, x) in samples:
        ref = _window_reference(a, b, (z, y, x), half, steps, w.g)
        got = f[:, :, z, y, x].cpu().numpy()
        assert np.max(np.abs(got - ref)) < 2e-6, (z, y, x, np.max(np.abs(got - ref)))
    d1 = sim.diagnostics()
    tot0 = d0["mass"][0] + d0["mass"][1]
    assert abs(d1["mass"][0] + d1["mass"][1] - tot0) / tot0 < 1e-6
    assert abs(d1["mass"][0] + d1["evaporated"] - d0["mass"][0]) / tot0 < 1e-6
    rho = sim.density(0)
    # the droplet is centred on ((N-1)/2)^3: mirror symmetry up to FP32 rounding
    for dim in (0, 1, 2):
        assert float((rho - torch.flip(rho, dims=(dim,))).abs().max()) < 1e-6
    del f, rho
    sim.close()
    torch.cuda.empty_cache()
