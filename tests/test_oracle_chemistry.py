"""Pins of the oracle's complex chemistry (ion model 4): tabulated
mobilities mu(E/N), drift-diffusion of positive and negative species,
electron attachment, channel target fractions and per-target elastic
recoil."""
import math

import numpy as np
import pytest

import oracle
from paper_1508_02892_amd import workloads as W

E_CH = 1.602176634e-19
ME = 9.1093837015e-31
NG = W.N_GAS_1ATM
DT = 2e-14


def _speed(eV):
    return np.sqrt(2 * E_CH * eV / ME)


def _flat_species(mu_pos=1e-3, mu_neg=2e-3, n_mu=8):
    return [{"charge": 1, "m_amu": W.HE_AMU, "en_lo_Td": 1.0, "en_hi_Td": 1000.0,
             "mu_m2_Vs": np.full(n_mu, mu_pos), "init_fraction": 1.0},
            {"charge": -1, "m_amu": W.O_AMU, "en_lo_Td": 1.0, "en_hi_Td": 1000.0,
             "mu_m2_Vs": np.full(n_mu, mu_neg), "init_fraction": 0.0}]


def _chem(n_macro=0, channels=None, species=None, **kw):
    return oracle.Oracle(W.small_chem(n_macro=n_macro,
                                      channels=channels if channels is not None else
                                      W.chem_channels(),
                                      species=species if species is not None else
                                      W.chem_species(), **kw))


def test_mobility_table_interpolates_in_log_field():
    o = _chem()
    sp = W.chem_species()
    x = np.logspace(0.0, 3.0, 64)
    for s in range(4):
        mu = sp[s]["mu_m2_Vs"]
        for k in (0, 5, 31, 62):
            E = x[k] * NG * 1e-21
            assert o.species_mobility(s, E) == pytest.approx(mu[k], rel=1e-11)
            # geometric midpoint: half way in ln(E/N)
            Em = math.sqrt(x[k] * x[k + 1]) * NG * 1e-21
            assert o.species_mobility(s, Em) == pytest.approx(0.5 * (mu[k] + mu[k + 1]),
                                                              rel=1e-11)
        # outside the table: the end values; E and -E alike
        assert o.species_mobility(s, 0.0) == mu[0]
        assert o.species_mobility(s, 0.5 * NG * 1e-21) == mu[0]
        assert o.species_mobility(s, 5e3 * NG * 1e-21) == mu[-1]
        assert o.species_mobility(s, -x[20] * NG * 1e-21) == o.species_mobility(s, x[20] * NG
                                                                                 * 1e-21)


@pytest.mark.parametrize("s,sign", [(0, 1.0), (1, -1.0)])
def test_species_centroid_drifts_with_its_charge(s, sign):
    # constant mobility tables: a positive pulse moves along E, a negative
    # one against it, both at mu E
    nc, gap, dt = 400, 1e-3, 1e-9
    o = oracle.Oracle(W.small_chem(n_macro=0, n_cells=nc, gap_m=gap, dt_s=dt,
                                   channels=W.chem_channels()[:2], species=_flat_species()))
    mu = 1e-3 if s == 0 else 2e-3
    z = np.arange(nc + 1) * gap / nc
    n = 1e17 * np.exp(-((z - 0.5e-3) / 0.05e-3) ** 2)
    E = np.full(nc + 1, 2e4)
    g = np.zeros(nc + 1)
    dV = np.full(nc + 1, gap / nc)
    dV[0] = dV[-1] = gap / nc / 2
    c0 = (z * n * dV).sum() / (n * dV).sum()
    for _ in range(1000):
        n, g, _ = o.fluid_species(s, n, g, E)
    c1 = (z * n * dV).sum() / (n * dV).sum()
    assert (c1 - c0) == pytest.approx(sign * mu * 2e4 * dt * 1000, rel=1e-6)


@pytest.mark.parametrize("s", [0, 3])
def test_species_conservation_and_wall_rule(s):
    o = _chem(n_cells=80)
    rng = np.random.default_rng(s)
    z = np.linspace(0, 1, 81)
    n = 1e17 * (0.2 + np.sin(np.pi * z) ** 2) * (1 + 0.1 * rng.random(81))
    E = 3e5 * (1 - 2 * z) + rng.normal(0, 1e4, 81)
    dz = o.derived()["dz"]
    dV = np.full(81, dz)
    dV[0] = dV[-1] = dz / 2
    n2, g, gw = o.fluid_species(s, n, np.zeros(81), E)
    assert abs(((n2 - n) * dV).sum() - DT * (gw[0] - gw[1])) <= 1e-9 * abs(DT * gw[0]) + 1e-3
    Z = W.chem_species()[s]["charge"]
    mu0, muN = o.species_mobility(s, E[0]), o.species_mobility(s, E[-1])
    # kept only when pointing into the wall
    assert gw[0] == pytest.approx(min(Z * mu0 * n[0] * E[0], 0.0), rel=1e-14)
    assert gw[1] == pytest.approx(max(Z * muN * n[-1] * E[-1], 0.0), rel=1e-14)
    # E points away from z = 0 at the left wall (E_0 > 0): positive ions
    # stay, negative ions leave into it
    assert (gw[0] < 0) == (Z < 0)


def test_attachment_removes_electrons_into_the_negative_ion():
    # sigma ~ 1/v: constant attachment frequency f N_g c on a fraction f of
    # the gas; every candidate attaches with P_max = 1 - exp(-f N_g c dt)
    Eg = W.energy_grid()
    c, f = 4e-14, 0.25
    sig = np.zeros_like(Eg)
    sig[1:] = c / _speed(Eg[1:])
    ch = [{"kind": "attachment", "threshold_eV": 0.0, "sigma_m2": sig, "product": 1,
           "target_fraction": f}]
    o = _chem(n_macro=20000, channels=ch, species=_flat_species(), v_amp_V=0.0, t_e0_eV=10.0,
              n_cells=64, gap_m=2e-3)
    steps = 12
    o.step(steps)
    cnt = o.counters()
    pm = 1 - math.exp(-f * NG * c * DT)
    n_att = int(cnt["coll"][0])
    pushed = int(cnt["pushed"])
    assert abs(n_att - pushed * pm) <= 5 * math.sqrt(pushed * pm * (1 - pm)) + 1
    # every lost electron is a negative ion; no wall losses this early
    assert cnt["absorbed"].sum() == 0
    live = (o.particles()["cell"] >= 0).sum()
    assert live == 20000 - n_att
    d = o.derived()
    dV = np.full(o.nn, d["dz"])
    dV[0] = dV[-1] = d["dz"] / 2
    neg = o.species(1)["n"]
    assert (neg * dV).sum() / d["w"] == pytest.approx(n_att, rel=1e-12)


def test_target_fractions_weight_the_channels():
    # two elastic channels of equal cross section on targets of fraction
    # 0.9 and 0.1: collisions split 9:1
    Eg = W.energy_grid()
    ch = [{"kind": "elastic", "threshold_eV": 0.0, "sigma_m2": np.full_like(Eg, 5e-20),
           "target_fraction": 0.9},
          {"kind": "elastic", "threshold_eV": 0.0, "sigma_m2": np.full_like(Eg, 5e-20),
           "target_fraction": 0.1, "target_mass_amu": W.O2_AMU}]
    o = _chem(channels=ch, species=_flat_species())
    n = 200_000
    v = _speed(10.0)
    ids = np.arange(n, dtype=np.uint32)
    chn, *_ = o.collide(np.full(n, 3, np.int32), np.full(n, 0.5), np.zeros(n), np.zeros(n),
                        np.full(n, v), ids, step=0)
    k0, k1 = (chn == 0).sum(), (chn == 1).sum()
    frac = k1 / (k0 + k1)
    assert abs(frac - 0.1) < 5 * math.sqrt(0.09 / (k0 + k1))
    # the total matches the null-collision probability of the full gas:
    # P_max nu(10 eV) / nu_max, nu_max at the table's top energy
    nu = NG * 5e-20 * v
    nu_max = NG * 5e-20 * _speed(Eg[-1])
    pm = (1 - math.exp(-nu_max * DT)) * nu / nu_max
    assert abs((k0 + k1) - n * pm) < 5 * math.sqrt(n * pm * (1 - pm))


def test_elastic_recoil_uses_the_target_mass():
    Eg = W.energy_grid()
    ch = [{"kind": "elastic", "threshold_eV": 0.0, "sigma_m2": np.full_like(Eg, 2e-18),
           "target_fraction": 0.5, "target_mass_amu": W.HE_AMU},
          {"kind": "elastic", "threshold_eV": 0.0, "sigma_m2": np.full_like(Eg, 2e-18),
           "target_fraction": 0.5, "target_mass_amu": W.O2_AMU}]
    o = _chem(channels=ch, species=_flat_species())
    n = 200_000
    rng = np.random.default_rng(3)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    v = _speed(10.0)
    chn, vx, vy, vz, _ = o.collide(np.full(n, 3, np.int32), np.full(n, 0.5), v * u[:, 0],
                                   v * u[:, 1], v * u[:, 2], np.arange(n, dtype=np.uint32),
                                   step=4)
    en = 0.5 * ME * (vx ** 2 + vy ** 2 + vz ** 2) / E_CH
    for k, m in ((0, W.HE_AMU), (1, W.O2_AMU)):
        hit = chn == k
        delta = 2 * ME / (m * 1.66053906660e-27)
        loss = 1 - en[hit] / 10.0
        assert abs(loss.mean() - delta) < 5 * delta * math.sqrt(1 / 3 / hit.sum())


def test_initial_state_is_neutral():
    o = _chem(n_macro=5000)
    g = o.grid()
    d = o.derived()
    ne = g["n_e"]
    np.testing.assert_array_equal(o.species(0)["n"], g["n_i"])
    assert np.allclose(g["n_i"], ne, rtol=1e-14, atol=0)
    for s in (1, 2, 3):
        assert not o.species(s)["n"].any()
    # no net charge: the field is the vacuum field V(0)/L (zero at phase 0)
    assert np.allclose(g["E"], 0.0, atol=1e-9 * d["w"])
