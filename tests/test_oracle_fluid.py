"""Pins of the oracle's ion fluid: drift-diffusion (Eqs 2.4-2.8) and the full
model (Eqs 2.3-2.4) against conservation, closed forms and the Boltzmann
steady state."""
import numpy as np
import pytest

import oracle
from paper_1508_02892_amd import workloads as W

E_CH = 1.602176634e-19
AMU = 1.66053906660e-27
KB = 1.380649e-23


def _fluid_disch(model, nc=64, gap=1e-3, dt=2e-14, **kw):
    return oracle.Oracle(W.small(ion_model=model, n_cells=nc, n_macro=0, gap_m=gap, dt_s=dt, **kw))


def test_wannier_factor_equal_masses():
    # Eq (2.8) with m_i = m_N: kappa = m_N / 4
    o = _fluid_disch(0)
    assert o.derived()["kappa"] == pytest.approx(W.HE_AMU * AMU / 4, rel=1e-14)


@pytest.mark.parametrize("model", [0, 1])
def test_conservation_telescopes_to_wall_fluxes(model):
    o = _fluid_disch(model, nc=80)
    d = o.derived()
    rng = np.random.default_rng(model)
    z = np.linspace(0, 1, 81)
    ni = 1e17 * (0.2 + np.sin(np.pi * z) ** 2) * (1 + 0.1 * rng.random(81))
    gam = rng.normal(0, 1e19, 81)
    E = 3e5 * (1 - 2 * z) + rng.normal(0, 1e4, 81)
    dV = np.full(81, d["dz"])
    dV[0] = dV[-1] = d["dz"] / 2
    before = (ni * dV).sum()
    ni2, gam2, gw = o.fluid(ni, gam, E)
    after = (ni2 * dV).sum()
    expect = 2e-14 * (gw[0] - gw[1])
    assert abs((after - before) - expect) <= 1e-9 * abs(expect) + 1e-12 * before


def test_dd_wall_flux_switch():
    o = _fluid_disch(0, nc=16)
    ni = np.full(17, 1e17)
    for E0, EN in [(-1e5, 1e5), (1e5, -1e5)]:
        E = np.linspace(E0, EN, 17)
        _, gam, gw = o.fluid(ni, np.zeros(17), E)
        assert gw[0] == pytest.approx(1e-3 * 1e17 * min(E0, 0.0))
        assert gw[1] == pytest.approx(1e-3 * 1e17 * max(EN, 0.0))


def test_dd_centroid_drifts_at_mobility_times_field():
    nc, gap, dt = 400, 1e-3, 1e-9
    o = _fluid_disch(0, nc=nc, gap=gap, dt=dt, mu_const=1e-3, t_gas_K=300.0)
    z = np.arange(nc + 1) * gap / nc
    ni = 1e17 * np.exp(-((z - 0.4e-3) / 0.05e-3) ** 2)
    E = np.full(nc + 1, 2e4)
    gam = np.zeros(nc + 1)
    dV = np.full(nc + 1, gap / nc)
    dV[0] = dV[-1] = gap / nc / 2
    c0 = (z * ni * dV).sum() / (ni * dV).sum()
    steps = 2000
    for _ in range(steps):
        ni, gam, _ = o.fluid(ni, gam, E)
    c1 = (z * ni * dV).sum() / (ni * dV).sum()
    assert (c1 - c0) == pytest.approx(1e-3 * 2e4 * dt * steps, rel=1e-6)


@pytest.mark.parametrize("nc", [32, 64])
def test_dd_relaxes_to_boltzmann_profile(nc):
    # Inward field E = E0 (1 - 2 z / L) closes both walls; with T ~ T_N the
    # zero-flux steady state is n ~ exp((e E0 / T)(z - z^2 / L)).
    gap, mu, E0 = 1e-3, 1e-3, 300.0
    D = mu * KB * 300.0 / E_CH
    dz = gap / nc
    dt = 0.2 * dz * dz / D
    o = _fluid_disch(0, nc=nc, gap=gap, dt=dt, mu_const=mu)
    z = np.arange(nc + 1) * dz
    E = E0 * (1 - 2 * z / gap)
    ni = np.full(nc + 1, 1e16)
    gam = np.zeros(nc + 1)
    steps = int(2 * gap * gap / D / dt)
    for _ in range(steps):
        ni, gam, _ = o.fluid(ni, gam, E)
    T = KB * 300.0
    exact = np.exp(E_CH * E0 / T * (z - z * z / gap))
    dV = np.full(nc + 1, dz)
    dV[0] = dV[-1] = dz / 2
    exact *= (ni * dV).sum() / (exact * dV).sum()
    err = np.abs(ni - exact).max() / exact.max()
    assert err < 0.02 * (32 / nc) ** 2
    # no odd/even checkerboard: second differences stay smooth
    dd = np.abs(np.diff(ni[1:-1], 2)).max() / ni.max()
    assert dd < 0.05 * (32 / nc) ** 2


def test_full_fluid_relaxes_in_closed_form():
    # Uniform n, E, nu, T: Eq (2.3) reduces to
    # G^{k+1/2} = r G^{k-1/2} + e E n dt / (M (1 + nu dt / 2)),
    # r = (1 - nu dt/2) / (1 + nu dt/2), fixed point mu n E with mu = e/(M nu).
    nc, dt, nu = 64, 2e-11, 3e9
    o = _fluid_disch(1, nc=nc, dt=dt, nu_const=nu)
    M = W.HE_AMU * AMU
    n0, E0 = 1e17, 1e5
    ni = np.full(nc + 1, n0)
    gam = np.zeros(nc + 1)
    E = np.full(nc + 1, E0)
    r = (1 - nu * dt / 2) / (1 + nu * dt / 2)
    drive = E_CH * E0 * n0 * dt / (M * (1 + nu * dt / 2))
    g = 0.0
    for k in range(40):
        ni2, gam, _ = o.fluid(ni, gam, E)
        g = r * g + drive
        assert gam[nc // 2] == pytest.approx(g, rel=1e-12), k
    mu = E_CH / (M * nu)
    assert abs(gam[nc // 2] / (mu * n0 * E0) - 1) < 2 * abs(r) ** 40 + 1e-12


def test_full_fluid_drift_diffusion_limit():
    nc, nu = 32, 3e9
    dt = 20.0 / nu
    o = _fluid_disch(1, nc=nc, dt=dt, nu_const=nu)
    M = W.HE_AMU * AMU
    ni = np.full(nc + 1, 1e17)
    E = np.full(nc + 1, 1e5)
    gam = np.zeros(nc + 1)
    for _ in range(200):
        _, gam, _ = o.fluid(ni, gam, E)
    assert gam[nc // 2] == pytest.approx(E_CH / (M * nu) * 1e17 * 1e5, rel=1e-10)
