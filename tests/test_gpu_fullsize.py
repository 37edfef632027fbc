"""Parity at the full workload sizes, in the launch configuration bench.py times.

128^3 droplet and 64x64x512 film: the whole lattice against the oracle over
1000 steps, in FP64 (rounding-order bars), FP32S and FP16N (storage bars).
512^3 droplet: sampled nodes against the oracle run on a window around each
sample (the state at a node after t steps depends only on nodes within 2t:
one hop for the pull, one for the force stencil), plus whole-lattice
properties (sink mass bookkeeping, mirror symmetry of the centred droplet).

Bars (from one storage rounding per step, accumulated over the run):
  FP64   populations within 1e-12 of max|f|; masses (against the exactly
         rounded sum of the oracle's densities) and E within 1e-13 of the
         total mass; z_I within 1e-9, R_I within 1e-10;
  FP32S  |drho|_inf <= 1e-5; total-mass and M^A + E drift <= 1e-6 of the
         total (the FP32 tolerance of the method's precision pattern);
         z_I within 0.01;
  FP16N  |drho|_inf <= 1e-3; drifts <= 1e-3; z_I within 0.1 (the FP16
         storage bars).
"""
import math

import numpy as np
import pytest
import torch

import lbinputs as li
from oracle.oracle import PSI_RHO, SINK_FACES, SINK_NONE, SINK_ZMAX, Oracle, OracleParams

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1701_03637_amd as lb
    lb.load_library()
    return lb


def _sim(lb, w, precision):
    return lb.Sim(lb.make_params(w.nx, w.ny, w.nz, wall_z=w.wall_z, g=w.g, psi=w.psi, precision=precision,
                                 sink=w.sink, rho_h=w.rho_h, shift=w.shift))


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


CONFIG_STEPS = 1000


@pytest.fixture(scope="module", params=["droplet_128", "film_deep"])
def config_run(request):
    """The oracle over 1000 steps of the 128^3 droplet or the 64x64x512 film
    (the two 2M-node configurations), from the workload's initial densities."""
    w = getattr(li, request.param)()
    orc = Oracle(OracleParams(w.nx, w.ny, w.nz, wall_z=w.wall_z, g=w.g, psi=PSI_RHO,
                              sink=SINK_FACES if w.sink == "faces" else SINK_ZMAX, rho_h=w.rho_h))
    a, b = w.densities()
    orc.init_from_density(a, b)
    d0 = orc.diagnostics()
    orc.step(CONFIG_STEPS)
    rho = orc.density()
    # masses of the oracle's field, rounded once: its own serial sum over
    # 2M nodes of largely equal densities carries correlated rounding of a
    # few 1e-7
    mass = tuple(math.fsum(r.ravel()) for r in rho)
    out = dict(w=w, a=a, b=b, d0=d0, d=orc.diagnostics(), pops=orc.populations(), rho=rho, mass=mass)
    del orc
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32s", "fp16n", "fp16nf"])
def test_config_1000_steps_against_oracle(lb, config_run, precision):
    w = config_run["w"]
    sim = _sim(lb, w, precision)
    sim.init_from_density(config_run["a"], config_run["b"])
    sim.step(CONFIG_STEPS)
    do, dg = config_run["d"], sim.diagnostics()
    tot = config_run["d0"]["mass"][0] + config_run["d0"]["mass"][1]
    assert dg["step"] == do["step"] == CONFIG_STEPS
    if precision == "fp64":
        ref = config_run["pops"]
        err = float((sim.populations().cpu() - torch.from_numpy(ref)).abs().max())
        assert err <= 1e-12 * np.max(np.abs(ref)), err
        for c in range(2):
            assert abs(dg["mass"][c] - config_run["mass"][c]) <= 1e-13 * tot, (c, dg["mass"][c] - config_run["mass"][c])
        assert abs(dg["evaporated"] - do["evaporated"]) <= 1e-13 * tot
        if w.init == "film":
            assert abs(dg["z_interface"] - do["z_interface"]) <= 1e-9
        else:
            assert abs(dg["r_droplet"] - do["r_droplet"]) <= 1e-10
    else:
        bar_rho, bar_z, bar_m = {"fp32s": (1e-5, 0.01, 1e-6), "fp16n": (1e-3, 0.1, 1e-3), "fp16nf": (1e-3, 0.1, 1e-3)}[precision]
        drho = float(np.max(np.abs(sim.density(0).cpu().numpy() - config_run["rho"][0])))
        m0 = config_run["d0"]["mass"]
        drift = abs(dg["mass"][0] + dg["mass"][1] - (m0[0] + m0[1])) / tot
        drift_ae = abs(dg["mass"][0] + dg["evaporated"] - m0[0]) / tot
        print(f"{w.name} {precision}: max |drho_A| = {drho:.3e}, mass drift {drift:.2e}, M^A + E drift {drift_ae:.2e}")
        assert drho <= bar_rho, drho
        assert drift <= bar_m and drift_ae <= bar_m
        if w.init == "film":
            assert abs(dg["z_interface"] - do["z_interface"]) <= bar_z
    sim.close()
    torch.cuda.empty_cache()


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


@pytest.mark.parametrize("precision,tol", [("fp32s", 2e-6), ("fp16n", 1e-4), ("fp16nf", 1e-4), ("fp64", 1e-12)])
def test_droplet512_sampled_and_properties(lb, precision, tol):
    """The 512^3 droplet in FP32S, in its FP16 variant (FP16N) and in FP64.
    Sampled populations against oracle windows: FP32S within 2e-6 (absolute;
    one rounding of deviations below 0.25 per step), FP16N within 1e-4 (FP16
    rounds the moving deviations, below 0.05, to 2^-11 of themselves), FP64
    within 1e-12 (summation order)."""
    w = li.droplet_512()
    steps = 3
    sim = _sim(lb, w, precision)
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
        assert np.max(np.abs(got - ref)) < tol, (z, y, x, np.max(np.abs(got - ref)))
    d1 = sim.diagnostics()
    tot0 = d0["mass"][0] + d0["mass"][1]
    bar_m = 1e-13 if precision == "fp64" else 1e-6
    assert abs(d1["mass"][0] + d1["mass"][1] - tot0) / tot0 < bar_m
    assert abs(d1["mass"][0] + d1["evaporated"] - d0["mass"][0]) / tot0 < bar_m
    rho = sim.density(0)
    # the droplet is centred on ((N-1)/2)^3: mirror symmetry up to storage
    # rounding
    for dim in (0, 1, 2):
        assert float((rho - torch.flip(rho, dims=(dim,))).abs().max()) < tol / 2
    del f, rho
    sim.close()
    torch.cuda.empty_cache()


def test_full_batch64_against_oracle_and_separate_runs(lb):
    """All 64 boxes of the batch workload (48^3..156^3, 74 M nodes) in one
    context, FP32S, 4 steps in the bench's launch configuration: every box
    bitwise against the same box stepped alone, and against the FP64 oracle
    (populations within 2e-6 of max|f|, the FP32S bar; M^A + E within 1e-6 of
    the total)."""
    ws = li.batch64()
    params = [lb.make_params(w.nx, w.ny, w.nz, g=w.g, psi=w.psi, precision="fp32s", sink=w.sink, rho_h=w.rho_h)
              for w in ws]
    batch = lb.Sim(params)
    batch.set_graph(2)
    for k, w in enumerate(ws):
        a, b = w.densities()
        batch.init_from_density(a, b, inst=k)
    steps = 4
    batch.step(steps)
    worst = 0.0
    for k, w in enumerate(ws):
        a, b = w.densities()
        got = batch.populations(inst=k)
        one = lb.Sim(params[k])
        one.init_from_density(a, b)
        one.step(steps)
        assert torch.equal(got, one.populations()), f"instance {k} ({w.nx}^3)"
        one.close()
        orc = Oracle(OracleParams(w.nx, w.ny, w.nz, g=w.g, psi=PSI_RHO, sink=SINK_FACES, rho_h=w.rho_h))
        orc.init_from_density(a, b)
        orc.step(steps)
        ref = orc.populations()
        err = float(np.max(np.abs(got.cpu().numpy() - ref))) / float(np.max(np.abs(ref)))
        worst = max(worst, err)
        assert err <= 2e-6, (k, w.nx, err)
        dg, do = batch.diagnostics(inst=k), orc.diagnostics()
        tot = do["mass"][0] + do["mass"][1]
        assert abs(dg["mass"][0] + dg["evaporated"] - (do["mass"][0] + do["evaporated"])) <= 1e-6 * tot, k
        del orc, got, ref
    print(f"64 boxes: worst population error {worst:.2e} of max|f|")
    batch.close()
    torch.cuda.empty_cache()

