"""The GPU path reproduces the paper's physics with its own parameters
(psi = 1 - exp(-rho), g = 3.6, tau = 1, FP64 storage).

- Sec. III B: a 4x4x128 film equilibrated without the sink, then evaporating
  towards rho_H in {0.035, 0.03, 0.02} for 10^6 steps: (x_H - d0 - x_I)^2 is
  linear in t with slope 2K (sign-fixed Eq. (xt)). With rho_H = 0.045 above
  the minority density the same boundary condenses vapour onto the film
  (Sec. II C, Sec. IV outlook): K < 0 and the film grows.
- Sec. III C: surface tension from static droplets (Laplace test), then a small
  evaporating droplet, and a small droplet growing by condensation, against
  RK4 solutions of the sign-fixed Eqs. (mass-dfsum-sim) and (drop-r-df4).
"""
import math

import numpy as np
import pytest
import torch

import lbinputs as li
from oracle import analytic as an

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def lb():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1701_03637_amd as lb
    lb.load_library()
    return lb


@pytest.fixture(scope="module")
def film_state(lb):
    """Equilibrated paper film (sink off), as FP64 populations."""
    p = lb.make_params(4, 4, 128, wall_z=True, g=3.6, psi="exp", precision="fp64")
    sim = lb.Sim(p)
    sim.set_graph(1000)
    a, b = li.film(4, 4, 128, 64)
    sim.init_from_density(a, b)
    sim.step(200000)
    f = sim.populations()
    ra = sim.density(0)[:, 0, 0].cpu().numpy()
    rb = sim.density(1)[:, 0, 0].cpu().numpy()
    return f, ra, rb


def test_film_coexistence_gpu(film_state):
    f, ra, rb = film_state
    rho_ma, rho_mi = ra[20:44].mean(), ra[84:108].mean()
    assert abs(rho_mi - 0.036) < 0.001 and abs(rho_ma - 0.704) < 0.006, (rho_ma, rho_mi)


@pytest.mark.parametrize("rho_h", [0.035, 0.03, 0.02, 0.045])
def test_film_sqrt_t_law_paper_length(lb, film_state, rho_h):
    f, ra, rb = film_state
    rho_ma, rho_mi, rho_t = ra[20:44].mean(), ra[84:108].mean(), ra[100] + rb[100]
    p = lb.make_params(4, 4, 128, wall_z=True, g=3.6, psi="exp", precision="fp64")
    sim = lb.Sim(p)
    sim.set_graph(1000)
    sim.init_from_populations(f)
    x0 = sim.diagnostics()["z_interface"]
    sim.set_sink("zmax", rho_h)
    T, nrec = 1_000_000, 40
    ts, xs = [], []
    for k in range(nrec):
        sim.step(T // nrec)
        ts.append((k + 1) * (T // nrec))
        xs.append(sim.diagnostics()["z_interface"])
    ts, xs = np.array(ts, float), np.array(xs)
    if rho_h < rho_mi:
        assert np.all(np.diff(xs) < 0), "film must evaporate"
    else:
        assert np.all(np.diff(xs) > 0), "film must grow by condensation"
    x_h = 127.0
    y = (x_h - xs) ** 2
    sel = ts > 0.1 * T
    p1, res, *_ = np.polyfit(ts[sel], y[sel], 1, full=True)
    r2 = 1 - res[0] / np.sum((y[sel] - y[sel].mean()) ** 2)
    ram = 0.5 * (rho_mi + rho_h)
    D = an.diffusion_small_gradient(ram, rho_t - ram, 3.6, "exp")
    K = an.film_rate_constant(D, rho_ma, rho_mi, rho_h)
    ratio = p1[0] / (2 * K)
    print(f"rho_H={rho_h}: x0={x0:.3f} x_I(1e6)={xs[-1]:.3f} slope/2K={ratio:.4f} R2={r2:.6f}")
    assert r2 > 0.999
    # rho_mi - rho_H is only 0.0011 at rho_H = 0.035, so a 1e-4 uncertainty of
    # the minority density moves K by ~9%: that case gets a wider band. The
    # condensing film's vapour (mean rho_A ~ 0.04) is the furthest from
    # symmetric composition, where Eq. (diffu-t-1)'s small-gradient D^c
    # overstates the measured decay rate of composition waves (by 20% at
    # (0.036, 0.704)); slope/2K falls with the vapour's rho_A across all four
    # cases (0.94, 0.90, 0.875, 0.87), so it shares the wider band.
    assert abs(ratio - 1) < (0.15 if rho_h in (0.035, 0.045) else 0.10)


@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
def test_diffusion_into_bath_gpu(lb, precision):
    """Sec. III A on the GPU: the diffusing component invades a box of its
    partner (rho = 0.7) from an evaporation boundary held at rho_H = 0.001,
    as the finite-difference solution of Fick's second law with the
    coefficient of Eq. (diffu-t-1) predicts (the bar of the oracle pin: 0.5%
    of rho_H)."""
    nz, rho_h, T = 125, 0.001, 8000
    sim = lb.Sim(lb.make_params(4, 4, nz, wall_z=True, g=3.6, psi="exp", precision=precision, sink="zmax",
                                rho_h=rho_h, shift=(0.0, 0.7)))
    sim.init_from_density(np.zeros((nz, 4, 4)), np.full((nz, 4, 4), 0.7))
    sim.step(T)
    ra = sim.density(0).cpu().numpy()
    u = an.fick_bath_fd(nz, rho_h, an.diffusion_small_gradient(0.5 * rho_h, 0.7, 3.6, "exp"), T)
    err = np.max(np.abs(ra[:, 0, 0] - u)) / rho_h
    print(f"{precision}: max |rho_A - Fick| = {err:.2e} of rho_H")
    assert np.ptp(ra, axis=(1, 2)).max() < (1e-15 if precision == "fp64" else 1e-9)
    assert err < 0.005


@pytest.fixture(scope="module")
def surface_tension(lb):
    """gamma from static droplets: P_in - P_out = 2 gamma / R, with the
    bulk pressure P = c_s^2 (rhoA + rhoB) + c_s^2 g psiA psiB (continuum limit
    of the Shan-Chen force with the weights of Eq. (sc)). The minority phase
    needs ~L^2/D ~ 3.4e4 steps of a 64^3 box to reach the Laplace-shifted
    coexistence, so each droplet relaxes 6e4 steps."""
    n = 64
    inv_r, dp = [], []
    c = (n - 1) / 2
    zz, yy, xx = np.meshgrid(*(np.arange(n) - c,) * 3, indexing="ij")
    r = np.sqrt(xx ** 2 + yy ** 2 + zz ** 2)
    for R0 in (10.0, 12.0, 14.0, 16.0):
        sim = lb.Sim(lb.make_params(n, n, n, g=3.6, psi="exp", precision="fp32s", shift=(0.04, 0.70)))
        sim.set_graph(100)
        a, b = li.droplet(n, n, n, R0)
        sim.init_from_density(a, b)
        sim.step(60000)
        ra, rb = sim.density(0).cpu().numpy(), sim.density(1).cpu().numpy()
        P = CS2 * (ra + rb) + CS2 * 3.6 * (1 - np.exp(-ra)) * (1 - np.exp(-rb))
        inside, outside = r < 5, r > 28
        # Equimolar radius from the excess of component A over the measured
        # outside bulk: a fixed-threshold phase field would count the
        # Laplace-raised vapour minority of the whole box as droplet volume.
        a_in, a_out = ra[inside].mean(), ra[outside].mean()
        V = (ra - a_out).sum() / (a_in - a_out)
        R = (3 * V / (4 * math.pi)) ** (1 / 3)
        assert R + 6 < 28, R
        p_in = P[inside].mean()
        p_out = P[outside].mean()
        inv_r.append(1 / R)
        dp.append(p_in - p_out)
        sim.close()
    slope, icpt = np.polyfit(inv_r, dp, 1)
    return slope / 2, icpt, inv_r, dp


def test_laplace_law(surface_tension):
    gamma, icpt, inv_r, dp = surface_tension
    print(f"gamma={gamma:.5f} intercept={icpt:.2e} 1/R={np.round(inv_r, 4)} dp={np.round(dp, 6)}")
    assert gamma > 0
    fit = np.polyval([2 * gamma, icpt], inv_r)
    assert np.max(np.abs(fit - dp)) < 0.05 * max(dp)   # linear in 1/R
    assert abs(icpt) < 0.05 * max(dp)                  # through the origin


def test_droplet_shrinks_like_the_radius_odes(lb, surface_tension):
    gamma = surface_tension[0]
    n, R0, RH, rho_h = 64, 16.0, 31.0, 0.02
    p = lb.make_params(n, n, n, g=3.6, psi="exp", precision="fp64", sink="none", rho_h=rho_h, sink_radius=RH,
                       phi_delta=(0.675, -0.675))
    sim = lb.Sim(p)
    sim.set_graph(100)
    a, b = li.droplet(n, n, n, R0)
    sim.init_from_density(a, b)
    sim.step(4000)
    ra = sim.density(0).cpu().numpy()
    rb = sim.density(1).cpu().numpy()
    c = n // 2
    rho_ma0 = ra[c - 2:c + 2, c - 2:c + 2, c - 2:c + 2].mean()
    zz, yy, xx = np.meshgrid(*(np.arange(n) - (n - 1) / 2,) * 3, indexing="ij")
    r = np.sqrt(xx ** 2 + yy ** 2 + zz ** 2)
    shell = (r > 27) & (r < 30)
    rho_mi0 = ra[shell].mean()
    rho_t = (ra + rb)[shell].mean()
    sim.set_sink("sphere", rho_h, RH)
    r_start = sim.diagnostics()["r_droplet"]
    ts, rs = [0.0], [r_start]
    for k in range(60):
        sim.step(500)
        d = sim.diagnostics()
        ts.append(500.0 * (k + 1))
        rs.append(d["r_droplet"])
        if d["r_droplet"] < 8:
            break
    ts, rs = np.array(ts), np.array(rs)
    ram = 0.5 * (rho_mi0 + rho_h)
    D = an.diffusion_small_gradient(ram, rho_t - ram, 3.6, "exp")
    d0 = 2.5
    t_plain, r_plain = an.rk4(lambda R: an.droplet_rate_plain(R, RH, d0, D, rho_ma0, rho_mi0, rho_h),
                              r_start, ts[-1], 50.0)
    t_lap, r_lap = an.rk4(lambda R: an.droplet_rate_laplace(R, RH, d0, D, r_start, gamma, rho_ma0, rho_mi0, rho_h),
                          r_start, ts[-1], 50.0)
    plain = np.interp(ts, t_plain, r_plain)
    lap = np.interp(ts, t_lap, r_lap)
    big = rs > 10.0   # the paper uses diameters above 20 only
    err_plain = np.max(np.abs(rs[big] - plain[big]))
    err_lap = np.max(np.abs(rs[big] - lap[big]))
    print(f"R: {np.round(rs[::4], 2)}\nplain: {np.round(plain[::4], 2)}\nlaplace: {np.round(lap[::4], 2)}")
    print(f"max |R - law| plain={err_plain:.3f} laplace={err_lap:.3f} gamma={gamma:.4f} D={D:.4f}")
    assert rs[-1] < r_start - 2, "droplet must evaporate"
    assert np.all(np.diff(rs) < 0)
    # The measured radius follows both laws to within ~6% of R while the
    # diameter exceeds 20; with D^c of Eq. (diffu-t-1) at the mean vapour
    # composition both laws run slightly fast (the same small-gradient
    # coefficient overestimates the measured decay rate of composition waves
    # at this asymmetric composition), the Laplace law, being faster, a
    # little more so.
    assert err_plain < 1.0
    assert err_lap < 1.0
    # The paper's claim for small droplets, on the shape of R(t), which does
    # not depend on D: the Laplace law's ratio of shrink rates between a small
    # and a larger radius is the closer one to the measured ratio.
    check_rate_shape(ts, rs, lambda R: an.droplet_rate_plain(R, RH, d0, D, rho_ma0, rho_mi0, rho_h),
                     lambda R: an.droplet_rate_laplace(R, RH, d0, D, r_start, gamma, rho_ma0, rho_mi0, rho_h),
                     10.0, 14.0)


def check_rate_shape(ts, rs, plain, laplace, r_small, r_large):
    """Ratio of the shrink rates at r_small and r_large: measured (central
    differences of R(t)) against each law's; the Laplace law must predict the
    faster relative shrinking of small droplets and be the closer one."""
    rate = -np.gradient(rs, ts)
    m = np.interp(-r_small, -rs, rate) / np.interp(-r_large, -rs, rate)
    p, q = plain(r_small) / plain(r_large), laplace(r_small) / laplace(r_large)
    print(f"rate({r_small})/rate({r_large}): measured {m:.4f}, plain law {p:.4f}, Laplace law {q:.4f}")
    assert q > p
    assert abs(m - q) <= abs(m - p)


def interface_radius(ra, r, mid):
    """Radius where the shell-averaged rho_A crosses mid (linear
    interpolation between 0.5-wide radial bins)."""
    k = (r / 0.5).astype(int).ravel()
    cnt = np.bincount(k)
    ok = cnt > 0   # the innermost bins hold no node
    prof = (np.bincount(k, weights=ra.ravel())[ok] / cnt[ok])
    rc = np.bincount(k, weights=r.ravel())[ok] / cnt[ok]
    i = int(np.argmax(prof < mid))
    assert i > 0 and prof[i] < mid <= prof[i - 1]
    return float(np.interp(mid, [prof[i], prof[i - 1]], [rc[i], rc[i - 1]]))


def test_droplet_grows_by_condensation(lb, surface_tension):
    """The sink set above the minority density (rho_H = 0.05 > rho_mi ~ 0.04)
    feeds vapour to the droplet: R(t) grows and follows the same sign-fixed
    laws, now with dM/dt > 0 (Sec. II C; the condensation case of the
    outlook in Sec. IV). R is the radial crossing of rho_A through the
    midpoint of the bulk densities: the phase-field volume of the
    diagnostics would also count the vapour's rise towards rho_H."""
    gamma = surface_tension[0]
    n, R0, RH, rho_h = 64, 12.0, 31.0, 0.05
    p = lb.make_params(n, n, n, g=3.6, psi="exp", precision="fp64", sink="none", rho_h=rho_h, sink_radius=RH,
                       phi_delta=(0.675, -0.675))
    sim = lb.Sim(p)
    sim.set_graph(100)
    a, b = li.droplet(n, n, n, R0)
    sim.init_from_density(a, b)
    sim.step(4000)
    ra = sim.density(0).cpu().numpy()
    rb = sim.density(1).cpu().numpy()
    c = n // 2
    rho_ma0 = ra[c - 2:c + 2, c - 2:c + 2, c - 2:c + 2].mean()
    zz, yy, xx = np.meshgrid(*(np.arange(n) - (n - 1) / 2,) * 3, indexing="ij")
    r = np.sqrt(xx ** 2 + yy ** 2 + zz ** 2)
    shell = (r > 27) & (r < 30)
    rho_mi0 = ra[shell].mean()
    rho_t = (ra + rb)[shell].mean()
    assert rho_h > rho_mi0 + 0.005
    mid = 0.5 * (rho_ma0 + rho_mi0)
    sim.set_sink("sphere", rho_h, RH)
    r_start = interface_radius(sim.density(0).cpu().numpy(), r, mid)
    ts, rs = [0.0], [r_start]
    for k in range(40):
        sim.step(500)
        assert sim.diagnostics()["nonfinite"] == 0
        ts.append(500.0 * (k + 1))
        rs.append(interface_radius(sim.density(0).cpu().numpy(), r, mid))
        if rs[-1] > 18:
            break
    ts, rs = np.array(ts), np.array(rs)
    ram = 0.5 * (rho_mi0 + rho_h)
    D = an.diffusion_small_gradient(ram, rho_t - ram, 3.6, "exp")
    d0 = 2.5
    t_plain, r_plain = an.rk4(lambda R: an.droplet_rate_plain(R, RH, d0, D, rho_ma0, rho_mi0, rho_h),
                              r_start, ts[-1], 50.0)
    t_lap, r_lap = an.rk4(lambda R: an.droplet_rate_laplace(R, RH, d0, D, r_start, gamma, rho_ma0, rho_mi0, rho_h),
                          r_start, ts[-1], 50.0)
    plain = np.interp(ts, t_plain, r_plain)
    lap = np.interp(ts, t_lap, r_lap)
    err_plain = np.max(np.abs(rs - plain))
    err_lap = np.max(np.abs(rs - lap))
    print(f"R: {np.round(rs[::4], 2)}\nplain: {np.round(plain[::4], 2)}\nlaplace: {np.round(lap[::4], 2)}")
    print(f"max |R - law| plain={err_plain:.3f} laplace={err_lap:.3f} gamma={gamma:.4f} D={D:.4f}")
    growth = (rs[-1] - r_start) / (plain[-1] - r_start)
    print(f"growth against the plain law: {growth:.3f}")
    assert rs[-1] > r_start + 2, "droplet must grow"
    # monotone once the sink's vapour front has crossed the 19-node gap to
    # the droplet (a diffusion time of ~19^2 / D ~ 3e3 steps; in the first
    # 500 steps the droplet still relaxes by a few 1e-3)
    assert np.all(np.diff(rs[ts >= 500]) > 0)
    # the same bar as the evaporating droplet: within one lattice unit; the
    # rate within the 20% by which the small-gradient D^c overstates the
    # composition decay rate at this vapour composition
    assert err_plain < 1.0
    assert 0.8 <= growth <= 1.05


def _wave_diffusion(lb, precision, nz, every, amp=1e-3, mean=0.37):
    """D from the decay of a composition wave along z: amplitude ~
    exp(-D k^2 t) (Eq. (fick2)), fitted over 8 intervals of `every` steps."""
    sim = lb.Sim(lb.make_params(4, 4, nz, g=0.9, psi="rho", precision=precision, shift=(mean, mean)))
    a, b = li.sinus(4, 4, nz, mean, mean, amp)
    sim.init_from_density(a, b)
    s = np.sin(2 * np.pi * np.arange(nz) / nz)
    amps, ts = [], []
    for k in range(9):
        if k:
            sim.step(every)
        ra = sim.density(0).cpu().numpy()[:, 0, 0]
        amps.append((ra - mean) @ s / (s @ s))
        ts.append(float(every * k))
    slope = np.polyfit(ts[2:], np.log(amps[2:]), 1)[0]
    return -slope / (2 * np.pi / nz) ** 2


# FP16S stores each population's deviation from a constant shift, and a step
# changes it by D k^2 of itself; FP16 resolves 2^-10 of it, so FP16S follows
# the decay only where D k^2 2^10 >= 1: waves shorter than ~47 nodes at
# D = 0.056. On the 128-node wave (D k^2 2^10 = 0.35) it stagnates; on a
# 32-node wave (2.2) it rounds each step's change by up to a quarter of
# itself and D comes out 1.1 % low, just outside the 1 % bar.
# The per-node forms store the moving values afresh each step relative to the
# node's own FP32 rest; there the limit is the size of those values, about
# 1e-7 for this wave of amplitude 1e-3: below FP16's smallest normal number
# (6.1e-5) FP16 keeps an absolute step of 6e-8, and FP16N's D comes out 3.6 %
# low at nz = 128 (0.8 % at nz = 32). FP16NF stores them times 2^12, in the
# normal range, and follows FP64 within 1e-4 on both waves.
@pytest.mark.parametrize("precision,nz,every,bar", [
    ("fp32s", 128, 500, 1e-3),
    ("fp16n", 32, 100, 1e-2),   # measured ratio 0.992
    ("fp16nf", 32, 100, 1e-2),  # measured ratio 1.00001
    ("fp16nf", 128, 500, 1e-2),  # measured ratio 1.0001
    pytest.param("fp16s", 32, 100, 1e-2, marks=pytest.mark.xfail(
        strict=True, reason="D k^2 2^10 = 2.2: FP16 rounding of ~2-ulp changes biases D (measured ratio 0.989)")),
    pytest.param("fp16n", 128, 500, 1e-2, marks=pytest.mark.xfail(
        strict=True, reason="moving deviations of ~1e-7 are FP16 subnormals, kept to 6e-8 (measured ratio 0.964)")),
    pytest.param("fp16s", 128, 500, 1e-2, marks=pytest.mark.xfail(
        strict=True, reason="D k^2 2^10 = 0.35: per-step changes below an FP16 ulp, the wave stagnates "
                            "(measured ratio 0.50)")),
])
def test_reduced_precision_diffusion_coefficient(lb, precision, nz, every, bar):
    """The diffusion coefficient measured through reduced-precision storage
    matches the FP64 run's on the same wave: within 0.1 % (FP32S) and 1 % (FP16
    forms, on waves they can resolve)."""
    d64 = _wave_diffusion(lb, "fp64", nz, every)
    dp = _wave_diffusion(lb, precision, nz, every)
    print(f"{precision} nz={nz}: D = {dp:.6f}, FP64 {d64:.6f}, ratio {dp / d64:.5f}")
    assert abs(dp / d64 - 1) < bar


def _vapour_diffusion(lb, ma, mb, nz=64, amp=1e-4, every=200):
    """D of a composition wave at mean composition (ma, mb) of the paper's
    fluid, FP64 on the GPU: amplitude ~ exp(-D k^2 t) (Eq. (fick2))."""
    sim = lb.Sim(lb.make_params(4, 4, nz, g=3.6, psi="exp", precision="fp64"))
    a, b = li.sinus(4, 4, nz, ma, mb, amp)
    sim.init_from_density(a, b)
    s = np.sin(2 * np.pi * np.arange(nz) / nz)
    amps, ts = [], []
    for k in range(9):
        if k:
            sim.step(every)
        amps.append((sim.density(0).cpu().numpy()[:, 0, 0] - ma) @ s / (s @ s))
        ts.append(every * k)
    return -np.polyfit(ts[2:], np.log(amps[2:]), 1)[0] / (2 * np.pi / nz) ** 2


@pytest.mark.parametrize("precision", ["fp32s", "fp16n", "fp16nf"])
def test_droplet_128_follows_the_radius_laws(lb, surface_tension, precision):
    """Sec. III C at half the paper's scale: a droplet of R0 = 32 in 128^3
    with a spherical sink at R_H = 63, rho_H = 0.02, equilibrated 8000 steps,
    then evaporating until R < 10 (the paper fits diameters above 20), in
    FP32S and in the per-node FP16 forms (FP16N, FP16NF).

    D is measured from a composition wave at the mean vapour composition
    (the small-gradient formula of Eq. (diffu-t-1) overstates it there).
    The laws are quasi-static: they hold once the vapour between droplet and
    sink has relaxed, a few diffusion times (R_H - R0)^2 / D after the sink
    is switched on, so they are integrated from the measured radius two
    diffusion times in. From there R(t) stays within one lattice unit (3 %
    of R0) of RK4 of both Eq. (mass-dfsum-sim) and Eq. (drop-r-df4) while
    R > 20 (measured 0.83 and 0.74). Below that the droplet shrinks faster
    than either law (at R ~ 10 both still give ~13); over the paper's range
    (diameter > 20) the Laplace law is the closer one, in its largest error
    (2.99 against 3.30) and on the D-independent shape of R(t) (the ratio of
    the shrink rates at R = 12 and R = 24). M^A + E = M^A(0) and the total
    mass hold to the storage's bar."""
    gamma = surface_tension[0]
    n, R0, RH, rho_h, d0 = 128, 32.0, 63.0, 0.02, 2.5
    p = lb.make_params(n, n, n, g=3.6, psi="exp", precision=precision, shift=(0.04, 0.70), sink="none",
                       rho_h=rho_h, sink_radius=RH, phi_delta=(0.675, -0.675))
    sim = lb.Sim(p)
    sim.set_graph(100)
    a, b = li.droplet(n, n, n, R0)
    sim.init_from_density(a, b)
    sim.step(8000)
    ra, rb = sim.density(0).cpu().numpy(), sim.density(1).cpu().numpy()
    c = n // 2
    rho_ma0 = ra[c - 2:c + 2, c - 2:c + 2, c - 2:c + 2].mean()
    zz, yy, xx = np.meshgrid(*(np.arange(n) - (n - 1) / 2,) * 3, indexing="ij")
    r = np.sqrt(xx ** 2 + yy ** 2 + zz ** 2)
    shell = (r > RH - 4) & (r < RH - 1)
    rho_mi0, rho_t = ra[shell].mean(), (ra + rb)[shell].mean()
    del ra, rb, zz, yy, xx, r
    sim.set_sink("sphere", rho_h, RH)
    d_start = sim.diagnostics()
    ts, rs = [0.0], [d_start["r_droplet"]]
    while rs[-1] > 9.5:
        sim.step(1000)
        d = sim.diagnostics()
        ts.append(ts[-1] + 1000)
        rs.append(d["r_droplet"])
        assert ts[-1] <= 200000, "droplet must evaporate"
    ts, rs = np.array(ts), np.array(rs)
    assert np.all(np.diff(rs) < 0)
    # mass bookkeeping over the whole run: FP32 storage within 1e-6 of the
    # total mass, FP16 storage within 1e-3
    m0 = d_start["mass"]
    tot = m0[0] + m0[1]
    drift = abs(d["mass"][0] + d["mass"][1] - tot) / tot
    drift_ae = abs(d["mass"][0] + d["evaporated"] - m0[0]) / tot
    print(f"{precision}: total-mass drift {drift:.2e}, M^A + E drift {drift_ae:.2e}")
    bar = 1e-6 if precision == "fp32s" else 1e-3
    assert drift <= bar and drift_ae <= bar
    ram = 0.5 * (rho_mi0 + rho_h)
    D = _vapour_diffusion(lb, ram, rho_t - ram)

    def plain(R):
        return an.droplet_rate_plain(R, RH, d0, D, rho_ma0, rho_mi0, rho_h)

    def laplace(R):
        return an.droplet_rate_laplace(R, RH, d0, D, rs[0], gamma, rho_ma0, rho_mi0, rho_h)

    t1 = 2 * (RH - rs[0]) ** 2 / D
    k1 = int(np.searchsorted(ts, t1))
    large, paper_range = rs[k1:] > 20.0, rs[k1:] > 10.0
    errs_large, errs = [], []
    for law in (plain, laplace):
        t_law, r_law = an.rk4(law, rs[k1], ts[-1] - ts[k1], 100.0)
        lawr = np.interp(ts[k1:] - ts[k1], t_law, r_law)
        errs_large.append(np.max(np.abs(rs[k1:] - lawr)[large]))
        errs.append(np.max(np.abs(rs[k1:] - lawr)[paper_range]))
        print(f"{law.__name__}: {np.round(lawr[::6], 2).tolist()}")
    print(f"R(t) every {6 * 1000} steps from t1 = {ts[k1]:.0f}: {np.round(rs[k1::6], 2).tolist()}")
    print(f"{precision}: {len(ts)} records, R {rs[0]:.2f} -> {rs[-1]:.2f} in {ts[-1]:.0f} steps; D = {D:.4f}; "
          f"from t1 max |R - law| while R > 20: plain {errs_large[0]:.3f}, Laplace {errs_large[1]:.3f}; "
          f"diameter > 20: plain {errs[0]:.3f}, Laplace {errs[1]:.3f}")
    assert max(errs_large) < 1.0
    assert errs[1] <= errs[0]
    check_rate_shape(ts, rs, plain, laplace, 12.0, 24.0)
    sim.close()
    torch.cuda.empty_cache()
