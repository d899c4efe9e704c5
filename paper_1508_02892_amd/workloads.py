"""Seeded synthetic workloads for the hybrid PIC/MCC discharge step.

This module only *defines inputs*: discharge parameters and electron-neutral
cross sections sampled on the uniform energy grid.  It contains none of the
method's arithmetic and is shared by the GPU binding, the CPU oracle, the tests
and the benchmark.

The paper's validation runs (helium at atmospheric pressure, mm-scale gaps,
Sec. III) use the XPDP1 helium cross sections, which are not available here;
analytic stand-ins with the same reaction set (elastic, excitation,
ionization; Table 1) replace them:

* elastic: 5e-20 m^2, constant;
* excitation: threshold 19.8 eV, linear rise to 5e-22 m^2 at 25 eV, then
  5e-22 * 25/E;
* ionization: threshold 24.6 eV, Lotz-like shape sigma = s0 p e ln(x) x^-p,
  x = E/24.6, p = 1/ln(120/24.6), whose maximum is exactly s0 = 3.5e-21 m^2 at
  E = 120 eV.
"""
from __future__ import annotations

import math

import numpy as np

HE_AMU = 4.002602
N_GAS_1ATM = 2.45e25

FP32, FP64 = 0, 1
ION_DD, ION_FULL, ION_DD_FIT, ION_FULL_FIT, ION_SPECIES = 0, 1, 2, 3, 4


def energy_grid(n_energy: int = 4096, inv_de_per_eV: float = 10.0) -> np.ndarray:
    """E_i = i / inv_de_per_eV [eV], i = 0 .. n_energy-1."""
    return np.arange(n_energy, dtype=np.float64) / inv_de_per_eV


def he_channels(n_energy: int = 4096, inv_de_per_eV: float = 10.0) -> list:
    """Synthetic analytic e-He cross sections (elastic, excitation, ionization)."""
    E = energy_grid(n_energy, inv_de_per_eV)
    el = np.full(n_energy, 5e-20)
    ex = np.zeros(n_energy)
    rise = (E >= 19.8) & (E < 25.0)
    ex[rise] = 5e-22 * (E[rise] - 19.8) / 5.2
    tail = E >= 25.0
    ex[tail] = 5e-22 * 25.0 / E[tail]
    iz = np.zeros(n_energy)
    p = 1.0 / math.log(120.0 / 24.6)
    above = E > 24.6
    x = E[above] / 24.6
    iz[above] = 3.5e-21 * p * math.e * np.log(x) * x ** (-p)
    return [
        {"kind": "elastic", "threshold_eV": 0.0, "sigma_m2": el},
        {"kind": "excitation", "threshold_eV": 19.8, "sigma_m2": ex},
        {"kind": "ionization", "threshold_eV": 24.6, "sigma_m2": iz},
    ]


def base_params(**over) -> dict:
    """Helium at 1 atm between plates; every field the discharge needs."""
    p = dict(
        precision=FP64, ion_model=ION_DD, n_cells=256, n_energy=4096, n_channels=3,
        sort_every=16, eedf_every=16, n_eedf_bins=128, n_macro=16384, seed=1,
        n_gas_m3=N_GAS_1ATM, t_gas_K=300.0, m_gas_amu=HE_AMU, gap_m=0.5e-3,
        v_amp_V=150.0, f_rf_Hz=13.56e6, phase_rad=0.0,
        n_e0_m3=1e17, t_e0_eV=2.0, load_lo=0.2, load_hi=0.8,
        gamma_see=0.1, e_sec_eV=2.0,
        m_ion_amu=HE_AMU, mu_const=1.0e-3, nu_const=3e9,
        dt_s=2e-14, inv_de_per_eV=10.0, eedf_emax_eV=50.0,
        power_W_m2=0.0, power_alpha=0.0,
        capacity=0,
    )
    p.update(over)
    if "channels" not in p:
        p["channels"] = he_channels(p["n_energy"], p["inv_de_per_eV"])
    p["n_channels"] = len(p["channels"])
    if not p["capacity"]:
        p["capacity"] = default_capacity(p["n_macro"])
    return p


def default_capacity(n_macro: int) -> int:
    """Room for growth by ionization and emission between compactions."""
    return int(n_macro + n_macro // 2 + 65536)


def c0(**over) -> dict:
    """Small plain case: 0.5 mm, 256 cells, 16,384 electrons, FP64, DD ions,
    150 V at 13.56 MHz, 2,000 steps."""
    return base_params(**over)


C0_STEPS = 2000


def c1(**over) -> dict:
    """Single large discharge: 1 mm, 2,048 cells, 8,388,608 FP32 electrons,
    full ion fluid with nu_m = 3e9 s^-1 (N_g / 2.45e25), 250 V, re-sort every
    16 steps, 20,000 steps."""
    p = dict(precision=FP32, ion_model=ION_FULL, n_cells=2048, n_macro=8388608, gap_m=1e-3,
             v_amp_V=250.0, nu_const=3e9 * (N_GAS_1ATM / 2.45e25), sort_every=16)
    p.update(over)
    return base_params(**p)


C1_STEPS = 20000


def cells_for_gap(gap_m: float) -> int:
    """256 cells at 0.3 mm rising to 4,096 at 2.0 mm, rounded to a multiple of 64."""
    return int(256 + 64 * round(3840.0 * (gap_m * 1e3 - 0.3) / 1.7 / 64.0))


def _sizes_to_total(x: np.ndarray, total: int, lo: int, hi: int) -> np.ndarray:
    n = np.clip(np.rint(x * (total / x.sum())), lo, hi).astype(np.int64)
    # distribute the remainder one particle at a time over the largest slots
    order = np.argsort(-n, kind="stable")
    i = 0
    while n.sum() != total:
        k = order[i % len(n)]
        step = 1 if n.sum() < total else -1
        if lo <= n[k] + step <= hi:
            n[k] += step
        i += 1
    return n


def c3(n_discharges: int = 64, total_electrons: int = 1 << 26, master_seed: int = 3) -> list:
    """Batched sweep: independent helium discharges, gap U(0.3, 2.0) mm, cells
    scaled to the gap, voltage U(100, 400) V, electrons log-uniform in
    [2^18, 2^23] rescaled to the stated total; Philox seed 1000 + d."""
    rng = np.random.default_rng(master_seed)
    gaps = rng.uniform(0.3e-3, 2.0e-3, n_discharges)
    volts = rng.uniform(100.0, 400.0, n_discharges)
    raw = np.exp(rng.uniform(math.log(2 ** 18), math.log(2 ** 23), n_discharges))
    sizes = _sizes_to_total(raw, total_electrons, 2 ** 18, 2 ** 23) if total_electrons else \
        np.rint(raw).astype(np.int64)
    out = []
    for d in range(n_discharges):
        out.append(base_params(precision=FP32, ion_model=ION_DD, gap_m=float(gaps[d]),
                               n_cells=cells_for_gap(float(gaps[d])), v_amp_V=float(volts[d]),
                               n_macro=int(sizes[d]), seed=1000 + d))
    return out


C3_STEPS = 5000


def scaled(p: dict, n_macro: int) -> dict:
    """Same discharge with a different superparticle count (weights follow Eq 1.2)."""
    q = dict(p)
    q["n_macro"] = int(n_macro)
    q["capacity"] = default_capacity(int(n_macro))
    return q


def c4_jobs(rate_per_s: float = 20.0, duration_s: float = 600.0, seed: int = 4,
            size_scale: float = 1.0, steps_range=(2000, 20000)) -> list:
    """Served stream: Poisson arrivals; each job is a discharge drawn like the
    batched sweep (sizes log-uniform in [2^18, 2^23] times size_scale) asking
    for a uniform number of steps in steps_range."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        gap = float(rng.uniform(0.3e-3, 2.0e-3))
        volt = float(rng.uniform(100.0, 400.0))
        n = int(round(math.exp(rng.uniform(math.log(2 ** 18), math.log(2 ** 23))) * size_scale))
        n = max(n, 64)
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        jobs.append({"arrival_s": t, "steps": steps,
                     "params": base_params(precision=FP32, ion_model=ION_DD, gap_m=gap,
                                           n_cells=cells_for_gap(gap), v_amp_V=volt,
                                           n_macro=n, seed=int(rng.integers(1, 2 ** 63)))})
    return jobs


def small(precision: int = FP64, ion_model: int = ION_DD, n_cells: int = 64,
          n_macro: int = 4096, **over) -> dict:
    """A few-second case for parity tests: several tiles and a ragged tail."""
    p = dict(precision=precision, ion_model=ion_model, n_cells=n_cells, n_macro=n_macro,
             gap_m=0.5e-3 * n_cells / 256.0)
    p.update(over)
    return base_params(**p)


# ---------------------------------------------------------------------------
# Auxiliary ion swarm (He+ in He): the isotropic-scattering cross section
# Q_m = Q_i + 2 Q_b of Sec. III as a rate coefficient k = Q_m g on the
# centre-of-mass energy eps = M_r g^2 / (2e).
# ---------------------------------------------------------------------------
AMU = 1.66053906660e-27
E_CHARGE = 1.602176634e-19


def he_ion_q(eps):
    """Q_i and Q_b [m^2] of He+ on He at centre-of-mass energy eps [eV] > 0."""
    eps = np.asarray(eps, np.float64)
    qi = 7.63e-20 / np.sqrt(eps)
    qb = 1e-19 / ((eps / 1000.0) ** 0.15 * (1.0 + eps / 1000.0) ** 0.25 * (1.0 + 5.0 / eps) ** 0.15)
    return qi, qb


def he_ion_rate(n_energy: int = 4096, inv_de_per_eV: float = 400.0) -> np.ndarray:
    """k(eps_i) = (Q_i + 2 Q_b) g on eps_i = i / inv_de_per_eV; at eps = 0 the
    limit (Q_i g is constant, Q_b g vanishes)."""
    Mr = HE_AMU * AMU / 2.0
    eps = np.arange(n_energy, dtype=np.float64) / inv_de_per_eV
    k = np.empty(n_energy)
    k[0] = 7.63e-20 * np.sqrt(2.0 * E_CHARGE / Mr)
    qi, qb = he_ion_q(eps[1:])
    g = np.sqrt(2.0 * E_CHARGE * eps[1:] / Mr)
    k[1:] = (qi + 2.0 * qb) * g
    return k


def swarm_params(e0_V_m, n_ions: int = 2048, precision: int = FP32, seed: int = 7,
                 **over) -> dict:
    """He+ swarms in He at 1 atm and 300 K, one per field value."""
    p = dict(precision=precision, n_ions=n_ions, seed=seed, n_gas_m3=N_GAS_1ATM, t_gas_K=300.0,
             m_ion_amu=HE_AMU, m_gas_amu=HE_AMU, t_i0_K=300.0, dt_s=5e-13, inv_de_per_eV=400.0,
             e0_V_m=np.asarray(e0_V_m, np.float64))
    p.update(over)
    if "rate_m3_s" not in p:
        p["rate_m3_s"] = he_ion_rate(4096, p["inv_de_per_eV"])
    return p


# The swarm measurement: 16 fields log-spaced over 1e5 .. 1e7 V/m (the range
# of Table 2), 2^20 He+ ions each, 2 ns to reach the stationary drift, then
# 2 ns averaged (Sec. II.C: "after several nanoseconds").
SWARM_WARM, SWARM_AVG = 4096, 4096


def swarm_bench(**over) -> dict:
    return swarm_params(np.logspace(5.0, 7.0, 16), n_ions=1 << 20, precision=FP32, seed=11,
                        **over)


# ---------------------------------------------------------------------------
# Complex chemistry: He with a 0.5 % O2-like molecular admixture.  Twelve
# synthetic channels (elastic on each target, six molecular excitations,
# dissociative-like attachment, three ionizations) and four drift-diffusion
# ion species with tabulated mobilities mu(E/N).
# ---------------------------------------------------------------------------
O2_AMU, O_AMU = 31.998, 15.999
X_O2 = 0.005  # molecular fraction of the gas
SPECIES_NAMES = ("He+", "He2+", "O2+", "O-")


def _lotz(E, thr, peak_eV, peak_m2):
    """Ionization shape s p e ln(x) x^-p, x = E/thr, peaking at peak_eV."""
    p = 1.0 / math.log(peak_eV / thr)
    out = np.zeros_like(E)
    above = E > thr
    x = E[above] / thr
    out[above] = peak_m2 * p * math.e * np.log(x) * x ** (-p)
    return out


def chem_channels(n_energy: int = 4096, inv_de_per_eV: float = 10.0) -> list:
    """The twelve channels; product = ion species index (0 He+, 1 He2+, 2 O2+, 3 O-)."""
    E = energy_grid(n_energy, inv_de_per_eV)
    fHe, fO2 = 1.0 - X_O2, X_O2
    ch = [{"kind": "elastic", "threshold_eV": 0.0, "sigma_m2": np.full(n_energy, 5e-20),
           "target_fraction": fHe, "target_mass_amu": HE_AMU},
          {"kind": "elastic", "threshold_eV": 0.0, "sigma_m2": np.full(n_energy, 9e-20),
           "target_fraction": fO2, "target_mass_amu": O2_AMU}]
    for k in range(6):
        thr = 0.2 * 50.0 ** (k / 5.0)
        peak = 2e-21 * 0.7 ** k
        sig = np.zeros(n_energy)
        rise = (E >= thr) & (E < 1.5 * thr)
        sig[rise] = peak * (E[rise] - thr) / (0.5 * thr)
        tail = E >= 1.5 * thr
        sig[tail] = peak * 1.5 * thr / E[tail]
        ch.append({"kind": "excitation", "threshold_eV": thr, "sigma_m2": sig,
                   "target_fraction": fO2, "target_mass_amu": O2_AMU})
    fwhm = 2.0
    att = 1e-22 * np.exp(-4.0 * math.log(2.0) * ((E - 6.5) / fwhm) ** 2)
    ch.append({"kind": "attachment", "threshold_eV": 0.0, "sigma_m2": att, "product": 3,
               "target_fraction": fO2, "target_mass_amu": O2_AMU})
    ch.append({"kind": "ionization", "threshold_eV": 24.6,
               "sigma_m2": _lotz(E, 24.6, 120.0, 3.5e-21), "product": 0,
               "target_fraction": fHe, "target_mass_amu": HE_AMU})
    ch.append({"kind": "ionization", "threshold_eV": 12.1,
               "sigma_m2": _lotz(E, 12.1, 80.0, 2.5e-20), "product": 2,
               "target_fraction": fO2, "target_mass_amu": O2_AMU})
    ch.append({"kind": "ionization", "threshold_eV": 18.0,
               "sigma_m2": _lotz(E, 18.0, 60.0, 1e-22), "product": 1,
               "target_fraction": fHe, "target_mass_amu": HE_AMU})
    return ch


def chem_species(seed: int = 2, n_mu: int = 64) -> list:
    """He+, He2+, O2+ and O- with mu(E/N) = mu0 (E/N)^-a on n_mu log-spaced
    points over 1..1000 Td, (mu0, a) drawn from a seeded generator, entries
    rounded to float32; He+ starts equal to the electron density."""
    rng = np.random.default_rng(seed)
    x = np.logspace(0.0, 3.0, n_mu)
    out = []
    for k, (name, Z, m) in enumerate(zip(SPECIES_NAMES, (1, 1, 1, -1),
                                         (HE_AMU, 2 * HE_AMU, O2_AMU, O_AMU))):
        mu0 = rng.uniform(0.8e-3, 2.5e-3)
        a = rng.uniform(0.0, 0.5)
        mu = (mu0 * x ** (-a)).astype(np.float32).astype(np.float64)
        out.append({"name": name, "charge": Z, "m_amu": m, "en_lo_Td": 1.0, "en_hi_Td": 1000.0,
                    "mu_m2_Vs": mu, "init_fraction": 1.0 if k == 0 else 0.0})
    return out


def c2(**over) -> dict:
    """Complex chemistry: 1 mm, 1,024 cells, 4,194,304 FP32 electrons, 300 V,
    twelve channels, four drift-diffusion ion species, 10,000 steps."""
    p = dict(precision=FP32, ion_model=ION_SPECIES, n_cells=1024, n_macro=4194304, gap_m=1e-3,
             v_amp_V=300.0, load_lo=0.2, load_hi=0.8, gamma_see=0.1,
             channels=chem_channels(), species=chem_species())
    p.update(over)
    return base_params(**p)


C2_STEPS = 10000


def small_chem(precision: int = FP64, n_cells: int = 64, n_macro: int = 4096, **over) -> dict:
    """A few-second complex-chemistry case for parity tests."""
    p = dict(precision=precision, ion_model=ION_SPECIES, n_cells=n_cells, n_macro=n_macro,
             gap_m=0.5e-3 * n_cells / 256.0, channels=chem_channels(), species=chem_species())
    p.update(over)
    return base_params(**p)
