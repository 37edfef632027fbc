"""The paper's evaporating droplet at its own scale (Sec. III C): 256^3 lattice,
R0 = 65, spherical evaporation boundary R_H = 127, rho_H = 0.03, 0.025 and
0.02 (the paper's three boundary densities), paper fluid (psi = 1 - exp(-rho),
g = 3.6, tau = 1), FP32-shifted storage.

R(t) is compared, while the diameter exceeds 20 (the paper's cut-off), with
RK4 solutions of the sign-fixed plain law (Eq. (mass-dfsum-sim)) and of the
law with Laplace pressure (Eq. (drop-r-df4)), gamma from the Laplace test of
test_gpu_physics. Each case is up to 7.5e5 steps of a 16.8 M-node lattice
(10-15 GPU-minutes): opt-in, LBSC_PAPER_SCALE=1 runs all three, or
LBSC_PAPER_SCALE=<rho_H> one of them; LBSC_PAPER_PRECISION picks the storage
form (default fp32s). FP16N reproduces the FP32S run at rho_H = 0.02; FP16S
does not (its vapour relaxation rounds away, see the transport limit of the
constant-shift FP16 form) and fails the radius-law check. rho_H = 0.03 drives the slowest
evaporation and stops at the step budget near R = 35, so its check covers
the large-R range only.
"""
import math
import os

import numpy as np
import pytest
import torch

import lbinputs as li
from oracle import analytic as an

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

CASES = [0.03, 0.025, 0.02]


def _enabled(rho_h):
    sel = os.environ.get("LBSC_PAPER_SCALE", "")
    return sel == "1" or (sel not in ("", "0") and abs(float(sel) - rho_h) < 1e-9)

GAMMA = 0.0483   # surface tension of the paper fluid, Laplace test on 64^3 (FP32S)


@pytest.mark.parametrize("rho_h", CASES)
def test_paper_scale_droplet_radius_laws(rho_h):
    if not _enabled(rho_h):
        pytest.skip("paper-scale run is opt-in (LBSC_PAPER_SCALE=1 or =<rho_H>)")
    import paper_1701_03637_amd as lb
    lb.load_library()
    n, R0, RH = 256, 65.0, 127.0
    precision = os.environ.get("LBSC_PAPER_PRECISION", "fp32s")
    p = lb.make_params(n, n, n, g=3.6, psi="exp", precision=precision, shift=(0.036, 0.708), sink="none",
                       rho_h=rho_h, sink_radius=RH, phi_delta=(0.672, -0.672))
    sim = lb.Sim(p)
    sim.set_graph(100)
    a, b = li.droplet(n, n, n, R0, rho_in=0.708, rho_out=0.036)
    sim.init_from_density(a, b)
    sim.step(5000)   # interface relaxation without the sink
    ra = sim.density(0).cpu().numpy()
    rb = sim.density(1).cpu().numpy()
    c = n // 2
    rho_ma0 = float(ra[c - 4:c + 4, c - 4:c + 4, c - 4:c + 4].mean())
    zz, yy, xx = np.meshgrid(*(np.arange(n, dtype=np.float32) - (n - 1) / 2,) * 3, indexing="ij")
    r = np.sqrt(xx ** 2 + yy ** 2 + zz ** 2)
    shell = (r > 100) & (r < 120)
    rho_mi0 = float(ra[shell].mean())
    rho_t = float((ra + rb)[shell].mean())
    del ra, rb, zz, yy, xx, r, shell
    sim.set_sink("sphere", rho_h, RH)
    d = sim.diagnostics()
    ts, rs = [0.0], [d["r_droplet"]]
    print(f"{precision} start: R={rs[0]:.2f} rho_ma={rho_ma0:.4f} rho_mi={rho_mi0:.4f} rho_t={rho_t:.4f}", flush=True)
    chunk = 10000
    for k in range(75):
        sim.step(chunk)
        d = sim.diagnostics()
        ts.append(chunk * (k + 1.0))
        rs.append(d["r_droplet"])
        print(f"t={ts[-1]:.0f} R={rs[-1]:.3f} E={d['evaporated']:.1f} nonfinite={d['nonfinite']}", flush=True)
        if rs[-1] < 10.0:
            break
    check_trajectory(np.array(ts), np.array(rs), rho_ma0, rho_mi0, rho_t, rho_h, RH, chunk, 75 * chunk)


def _law(rate, r0, t_end, radius):
    """RK4 of dR/dt = rate(R) from R(0) = r0 to t_end, continued (in tenths
    of t_end, up to 3 t_end) until R drops below radius."""
    ts, rs = an.rk4(rate, r0, t_end, 500.0)
    ts, rs = list(ts), list(rs)
    while rs[-1] >= radius and ts[-1] < 3 * t_end:
        t2, r2 = an.rk4(rate, rs[-1], 0.1 * t_end, 500.0)
        ts += [ts[-1] + t for t in t2[1:]]
        rs += list(r2[1:])
    return np.array(ts), np.array(rs)


def _t_at(tt, rr, radius):
    """First time R(t) crosses radius (linear interpolation)."""
    i = int(np.argmax(rr < radius))
    assert i > 0, "never reaches the radius"
    return float(np.interp(radius, [rr[i], rr[i - 1]], [tt[i], tt[i - 1]]))


def check_trajectory(ts, rs, rho_ma0, rho_mi0, rho_t, rho_h, RH, chunk, max_steps):
    """R(t) of the sink-driven droplet against both radius laws."""
    ram = 0.5 * (rho_mi0 + rho_h)
    D = an.diffusion_small_gradient(ram, rho_t - ram, 3.6, "exp")
    d0 = 2.5
    t_p, r_p = _law(lambda R: an.droplet_rate_plain(R, RH, d0, D, rho_ma0, rho_mi0, rho_h), rs[0], ts[-1], 15.0)
    t_l, r_l = _law(lambda R: an.droplet_rate_laplace(R, RH, d0, D, rs[0], GAMMA, rho_ma0, rho_mi0, rho_h),
                    rs[0], ts[-1], 15.0)
    plain = np.interp(ts, t_p, r_p)
    lap = np.interp(ts, t_l, r_l)
    big = rs > 10.0
    err_p = float(np.max(np.abs(rs[big] - plain[big])))
    err_l = float(np.max(np.abs(rs[big] - lap[big])))
    over20 = rs > 20.0
    err20_p = float(np.max(np.abs(rs[over20] - plain[over20])))
    err20_l = float(np.max(np.abs(rs[over20] - lap[over20])))
    print(f"rho_H = {rho_h}, {ts[-1]:.0f} steps")
    print(f"R:       {np.round(rs[::5], 2)}\nplain:   {np.round(plain[::5], 2)}\nlaplace: {np.round(lap[::5], 2)}")
    print(f"max |R - law| while R > 20: plain {err20_p:.2f}, Laplace {err20_l:.2f}; while the diameter exceeds 20: "
          f"plain {err_p:.2f}, Laplace {err_l:.2f} (D={D:.4f}, gamma={GAMMA})")
    # R grows by ~0.1 while the sink's depletion front forms, then shrinks
    # monotonically
    after = ts >= 2 * chunk
    assert np.all(np.diff(rs[after]) < 0), "the droplet must shrink monotonically"
    # both laws within 5% of R0 while R > 20
    assert err20_p < 0.05 * rs[0] and err20_l < 0.05 * rs[0]
    if rs[-1] < 15.0:
        # the time to reach R = 15 within 10% of both laws'
        t15, t15_p, t15_l = _t_at(ts, rs, 15.0), _t_at(t_p, r_p, 15.0), _t_at(t_l, r_l, 15.0)
        print(f"t(R = 15): {t15:.0f}; plain law {t15_p:.0f}, Laplace law {t15_l:.0f}")
        assert abs(t15 / t15_p - 1) < 0.10 and abs(t15 / t15_l - 1) < 0.10
        # the law with Laplace pressure is the closer one for small droplets
        # (the paper's point)
        assert err_l <= err_p
    else:
        # only the step budget may stop a run short of R = 15
        assert ts[-1] >= max_steps
