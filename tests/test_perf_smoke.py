"""Performance smoke tests: regression bands, not benchmarks.

CPU: the committed HBM counter record of the 512^3 FP32S step (the bench's
roofline.traffic) stays within 10 % of the byte model (2 x 19 x 4 B read and
written per node), its reads within 20 %.

GPU: the fused step on the 128^3 droplet, the 512^3 droplet and the 64-box
batch runs at no less than about two thirds of its measured fraction of the
8 TB/s HBM peak (algorithmic bytes over the step kernel's time, HIP events on
the library's stream). The bands catch a lost schedule, a spilling build or a
serialised launch; run-to-run and box-to-box spreads (a few percent) stay far
inside them.
"""
import json
import os

import pytest

import lbinputs as li

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PEAK_GBPS = 8000.0
B_PER_LU_FP32S = 304


def test_committed_traffic_record_is_near_the_byte_model():
    from paper_1701_03637_amd.build import kernel_hash
    with open(os.path.join(ROOT, "profiles", "traffic_droplet512_fp32s.json")) as fh:
        rec = json.load(fh)
    if rec["kernel_hash"] != kernel_hash():
        pytest.skip("the record was taken on other kernel sources (the bench reports no traffic then)")
    nodes = 512 ** 3
    # reads carry the halo rows, columns and chunk planes fetched again
    # (x1.12 measured); writes are the stores alone
    assert 1.0 <= rec["read_bytes"] / (nodes * B_PER_LU_FP32S / 2) <= 1.20
    assert 0.99 <= rec["write_bytes"] / (nodes * B_PER_LU_FP32S / 2) <= 1.01
    assert 1.0 <= rec["bytes_per_launch"] / (nodes * B_PER_LU_FP32S) <= 1.10


def _step_ms(torch, sim, steps, warmup):
    sim.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


# workload, steps, measured fraction of peak (bench runs on four boxes), band
SINGLE = [("droplet_128", 200, 0.55, 0.37), ("droplet_512", 20, 0.59, 0.40)]


@pytest.mark.gpu
@pytest.mark.parametrize("name,steps,measured,band", SINGLE)
def test_single_lattice_step_rate_band(name, steps, measured, band):
    import torch
    import paper_1701_03637_amd as lb
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    lb.load_library()
    w = getattr(li, name)()
    sim = lb.Sim(lb.make_params(w.nx, w.ny, w.nz, g=w.g, psi=w.psi, precision="fp32s", sink=w.sink,
                                rho_h=w.rho_h, shift=w.shift))
    a, b = w.densities()
    sim.init_from_density(a, b)
    del a, b
    ms = _step_ms(torch, sim, steps, 5)
    frac = w.nodes * B_PER_LU_FP32S / (ms * 1e-3) / 1e9 / PEAK_GBPS
    print(f"{w.name} fp32s: {ms:.4f} ms per step, {frac:.3f} of peak (measured {measured}, band {band})")
    sim.close()
    torch.cuda.empty_cache()
    assert frac >= band


@pytest.mark.gpu
def test_batch_step_rate_band():
    """The 64-box batch, default schedule, replayed as HIP graphs of 10
    steps (measured 0.50-0.54 of peak, depending on where its buffers land)."""
    import torch
    import paper_1701_03637_amd as lb
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    lb.load_library()
    ws = li.batch64()
    sim = lb.Sim([lb.make_params(w.nx, w.ny, w.nz, g=w.g, psi=w.psi, precision="fp32s", sink=w.sink,
                                 rho_h=w.rho_h) for w in ws])
    for k, w in enumerate(ws):
        a, b = w.densities()
        sim.init_from_density(a, b, inst=k)
    sim.set_graph(10)
    ms = _step_ms(torch, sim, 20, 10)
    nodes = sum(w.nodes for w in ws)
    frac = nodes * B_PER_LU_FP32S / (ms * 1e-3) / 1e9 / PEAK_GBPS
    print(f"batch64 fp32s: {ms:.4f} ms per step, {frac:.3f} of peak (band 0.33)")
    sim.close()
    torch.cuda.empty_cache()
    assert frac >= 0.33
