"""The allocation-free binding (lbsc_bind_static): the library's static
scratch array in place of a caller scratch buffer gives the same bits as
lbsc_bind, for two contexts bound to it in a row, the second smaller (it
takes the array over and must start from cleared accumulators), and the
first context is refused once the second owns the array."""
import numpy as np
import pytest
import torch

import lbinputs as li

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1701_03637_amd as lb
    lb.load_library()
    return lb


def _run(lb, n, static, precision, steps):
    p = lb.make_params(n, n, n, g=0.9, psi="rho", sink="faces", rho_h=0.03, precision=precision)
    sim = lb.Sim(p, static_scratch=static)
    a, b = li.droplet(n, n, n, 0.25 * n)
    sim.init_from_density(a, b)
    sim.step(steps)
    return sim


@pytest.mark.parametrize("precision", ["fp32s", "fp64"])
def test_static_scratch_matches_caller_scratch(lb, precision):
    first = None
    for n, steps in ((72, 23), (40, 11)):   # the second call smaller
        ref = _run(lb, n, False, precision, steps)
        got = _run(lb, n, True, precision, steps)
        assert torch.equal(got.populations(), ref.populations()), n
        dg, dr = got.diagnostics(), ref.diagnostics()
        assert dg["evaporated"] == dr["evaporated"] and dg["mass"] == dr["mass"], n
        assert dg["evaporated"] != 0.0
        got.step(3)
        ref.step(3)
        assert torch.equal(got.populations(), ref.populations()), n
        if first is None:
            first = got
        else:
            # the second context owns the array now
            with pytest.raises(lb.LbscError) as e:
                first.step(1)
            assert e.value.status == -2
        ref.close()
    first.close()
    got.close()


def test_static_scratch_refuses_a_context_too_large(lb):
    p = lb.make_params(300, 300, 300, precision="fp16n")   # about 70 MiB of scratch
    with pytest.raises(lb.LbscError) as e:
        lb.Sim(p, static_scratch=True)
    assert e.value.status == -1
