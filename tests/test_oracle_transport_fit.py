"""Pins of the oracle's fitted He+ transport (Tables 2 and 3): its logarithm
and exponential against numpy, the fits at points where they reduce to
closed forms, and the fitted ion fluids against the steady drift they must
reach in a uniform field."""
import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from paper_1508_02892_amd import workloads as W

E_CH = 1.602176634e-19
AMU = 1.66053906660e-27
E0 = 1.47e6  # Table 2 branch field [V/m]
U0 = 2e3  # Table 3 branch speed [m/s]


def _mu_table(E):
    a = abs(E)
    return 1e-3 * (1.18 - 0.185 * a / E0) if a < E0 else 1e-3 * 0.94 * np.power(E0 / a, 0.3)


def _nu_table(u):
    a = abs(u)
    return 1e10 * (2.07 + 0.88 * np.power(a / U0, 1.89)) if a < U0 else 1e10 * (1.54 + 1.36 * a / U0)


def test_ln_matches_numpy():
    xs = np.concatenate([np.logspace(-300, 300, 1201), np.linspace(0.5, 2.0, 1201),
                         [0.7071067811865476, 1.4142135623730951, 2.0, 4.0, 0.25]])
    for x in xs:
        ref = np.log(x)
        assert abs(oracle.fit_ln(x) - ref) <= 4.5e-16 * abs(ref) + 1e-300, x
    assert oracle.fit_ln(1.0) == 0.0
    assert oracle.fit_ln(2.0) == np.log(2.0)


def test_exp_matches_numpy():
    for y in np.concatenate([np.linspace(-700, 700, 4001), np.linspace(-1, 1, 401)]):
        ref = np.exp(y)
        assert abs(oracle.fit_exp(y) - ref) <= 4.5e-16 * ref, y
    assert oracle.fit_exp(0.0) == 1.0


@pytest.mark.parametrize("contract", [False, True])
def test_mobility_fit_closed_forms(contract):
    def mu(E):
        return oracle.mobility_fit(E, contract)
    assert mu(0.0) == pytest.approx(1.18e-3, rel=1e-15)
    assert mu(E0 / 2) == pytest.approx(1.0875e-3, rel=1e-15)
    assert mu(np.nextafter(E0, 0.0)) == pytest.approx(0.995e-3, rel=1e-15)
    # the high-field branch starts at E0 with 0.94, a jump of 0.055 down
    assert mu(E0) == pytest.approx(0.94e-3, rel=1e-15)
    # (1/1024)^0.3 = 1/8
    assert mu(1024 * E0) == pytest.approx(0.1175e-3, rel=1e-14)
    for E in [3e5, 2e6, 1e8]:
        assert mu(-E) == mu(E)


@pytest.mark.parametrize("contract", [False, True])
def test_mobility_fit_matches_table_everywhere(contract):
    for E in np.concatenate([np.linspace(0, 3 * E0, 301), np.logspace(2, 9, 141)]):
        assert oracle.mobility_fit(E, contract) == pytest.approx(_mu_table(E), rel=2e-15, abs=0), E


@pytest.mark.parametrize("contract", [False, True])
def test_nu_fit_closed_forms(contract):
    def nu(u):
        return oracle.nu_fit(u, contract)
    assert nu(0.0) == pytest.approx(2.07e10, rel=1e-15)
    assert nu(np.nextafter(U0, 0.0)) == pytest.approx(2.95e10, rel=1e-14)
    # the high-speed branch starts at u0 with 1.54 + 1.36, a jump of 0.05 down
    assert nu(U0) == pytest.approx(2.90e10, rel=1e-15)
    assert nu(2 * U0) == pytest.approx(4.26e10, rel=1e-15)
    for u in [500.0, 3e3, 1e5]:
        assert nu(-u) == nu(u)


def test_fits_agree_with_eq_2_6_at_low_speed():
    # The two tables describe one ion: at vanishing field and speed, Eq (2.6)
    # links them, e/(M mu(0)) = 2.04e10 against nu(0) = 2.07e10.
    M = W.HE_AMU * AMU
    assert E_CH / (M * oracle.mobility_fit(0.0)) == pytest.approx(oracle.nu_fit(0.0), rel=0.02)


@pytest.mark.parametrize("contract", [False, True])
def test_nu_fit_matches_table_everywhere(contract):
    for u in np.concatenate([np.linspace(0, 3 * U0, 301), np.logspace(-3, 6, 181)]):
        assert oracle.nu_fit(u, contract) == pytest.approx(_nu_table(u), rel=2e-15, abs=0), u


def _disch(model, nc=64, gap=1e-3, dt=2e-14, contract=False, **kw):
    return oracle.Oracle(W.small(ion_model=model, n_cells=nc, n_macro=0, gap_m=gap, dt_s=dt, **kw),
                         contract=contract)


@pytest.mark.parametrize("E", [4e5, 1.2e6, 3e6, 2e7])
def test_dd_fit_drift_in_uniform_field(E):
    # uniform density and field: no gradient, the interior flux is mu(E) n E
    o = _disch(W.ION_DD_FIT, nc=32)
    n = 3e17
    _, gam, gw = o.fluid(np.full(33, n), np.zeros(33), np.full(33, E))
    expect = _mu_table(E) * n * E
    assert np.allclose(gam[1:-1], expect, rtol=2e-15, atol=0)
    assert gw[0] == 0.0
    assert gw[1] == pytest.approx(expect, rel=2e-15)


def test_dd_fit_diffusion_uses_local_mobility():
    # Linear density in a uniform field: the central difference is exact, so
    # Gamma_j = mu n_j E - (mu T / e) dn/dz with T from Eq (2.8) at mu(E).
    nc, gap, E = 32, 1e-3, 2e6
    o = _disch(W.ION_DD_FIT, nc=nc, gap=gap)
    d = o.derived()
    z = np.arange(nc + 1) * gap / nc
    n = 1e17 * (1 + 2 * z / gap)
    _, gam, _ = o.fluid(n, np.zeros(nc + 1), np.full(nc + 1, E))
    mu = _mu_table(E)
    T = d["TN"] + d["kappa"] * (mu * E) ** 2
    expect = mu * n * E - mu * T / E_CH * (2e17 / gap)
    assert np.allclose(gam[1:-1], expect[1:-1], rtol=1e-12, atol=0)


@pytest.mark.parametrize("contract", [False, True])
@pytest.mark.parametrize("E", [1e6, 7e6])
def test_full_fit_reaches_steady_drift(E, contract):
    # In a uniform field and density the discrete Eq (2.3) has its fixed
    # point at u nu(u) = e E / M: one root below u0 (E = 1e6) and one above
    # (E = 7e6).
    nc, dt = 64, 2e-12
    o = _disch(W.ION_FULL_FIT, nc=nc, dt=dt, contract=contract)
    M = W.HE_AMU * AMU
    target = E_CH * E / M
    u_star = brentq(lambda u: u * _nu_table(u) - target, 1.0, 1e6, xtol=1e-14, rtol=1e-15)
    assert (u_star < U0) == (E < 2e6)
    n = np.full(nc + 1, 2e17)
    gam = np.zeros(nc + 1)
    Ev = np.full(nc + 1, E)
    for _ in range(1500):
        n, gam, _ = o.fluid(n, gam, Ev)
    mid = nc // 2
    assert gam[mid] / n[mid] == pytest.approx(u_star, rel=1e-10)


@pytest.mark.parametrize("contract", [False, True])
@pytest.mark.parametrize("model", [W.ION_DD_FIT, W.ION_FULL_FIT])
def test_fitted_models_conserve(model, contract):
    nc = 80
    o = _disch(model, nc=nc, contract=contract)
    d = o.derived()
    rng = np.random.default_rng(7 + model)
    z = np.linspace(0, 1, nc + 1)
    ni = 1e17 * (0.2 + np.sin(np.pi * z) ** 2) * (1 + 0.1 * rng.random(nc + 1))
    gam = rng.normal(0, 1e20, nc + 1)
    E = 3e6 * (1 - 2 * z) + rng.normal(0, 1e5, nc + 1)
    dV = np.full(nc + 1, d["dz"])
    dV[0] = dV[-1] = d["dz"] / 2
    before = (ni * dV).sum()
    ni2, _, gw = o.fluid(ni, gam, E)
    expect = 2e-14 * (gw[0] - gw[1])
    assert abs(((ni2 * dV).sum() - before) - expect) <= 1e-9 * abs(expect) + 1e-12 * before
