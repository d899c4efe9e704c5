// Plain CPU oracle for the 1D hybrid PIC/MCC discharge step of Eremin, Hemke &
// Mussenbrock, "A New Hybrid Scheme for Simulations of Highly Collisional
// RF-Driven Plasmas" (arXiv 1508.02892).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
// this file: it exists so that tests, the smoke check and the CPU-baseline leg
// of the benchmark can check the GPU library against an independent, slow,
// obviously-correct implementation.  It shares no code, header, table or
// constant generator with the GPU library.
//
// Field/fluid arithmetic is FP64.  The electron particle state and the Monte
// Carlo arithmetic use the scalar type P (float or double), selected at run
// time by the `precision` parameter.  Expressions are written in a fixed
// evaluation order and compiled with -ffp-contract=off; where a fused
// multiply-add is part of the definition it is written as std::fma.
//
// Parity status per function (pins live in tests/test_oracle_*.py):
//   philox4x32_10 ............ pinned (published known-answer vectors, rocRAND)
//   uniform maps .............. pinned (exact bit patterns)
//   initial load .............. pinned (exact charge, statistical moments)
//   field solve (Poisson) ..... pinned (Thomas vs dense solve, linear/parabolic
//                               closed forms, discrete Gauss law); the
//                               fixed-order solve within the conditioning
//                               bound of Thomas
//   push ...................... pinned (free streaming, uniform-field leapfrog)
//   null-collision MCC ........ pinned (binomial collision counts, channel
//                               fractions, energy bookkeeping, isotropy)
//   CIC deposit ............... pinned (exact total, single-node case)
//   DD ion fluid .............. pinned (conservation, centroid drift, Boltzmann
//                               steady state)
//   full ion fluid ............ pinned (closed-form relaxation, Thomas vs dense;
//                               fixed-order solve against Thomas)
//   fitted transport .......... pinned (closed-form points, numpy's power; the
//                               series log/exp within 1 ulp of numpy)
//   secondary emission ........ pinned (mean count, cosine law)
//   compaction + sort ......... pinned (equals a stable sort by cell)
//   run averages .............. pinned (free-streaming closed form of the
//                               accumulated deposit over levels 1..S; ion
//                               content fed by ionization)
//   literal sub-step order .... pinned (first-step difference = deposit of the
//                               new electrons; per-step charge deficit)
//   decision-locked replay .... pinned (its float run equals the plain float
//                               run; the double run follows every decision)
//   threaded particle loop .... pinned (bitwise equal runs on 1, 3, 8 threads)
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Physical constants (CODATA 2018).
// ---------------------------------------------------------------------------
constexpr double kE = 1.602176634e-19;      // elementary charge [C]
constexpr double kMe = 9.1093837015e-31;    // electron mass [kg]
constexpr double kEps0 = 8.8541878128e-12;  // vacuum permittivity [F/m]
constexpr double kKb = 1.380649e-23;        // Boltzmann constant [J/K]
constexpr double kAmu = 1.66053906660e-27;  // atomic mass unit [kg]
constexpr double kPi = 3.14159265358979323846;

constexpr int kMaxChannels = 16;
constexpr int kSphereTries = 64;     // rejection-loop bound (probability of
                                     // exhausting it is (1-pi/4)^64 ~ 1e-43)
constexpr int64_t kSeeMaxPerSide = 4096;

// Arithmetic modes.  By default the oracle is the plain reference: the
// tridiagonal systems of the field (Sec. II.D) and of Eq (2.3) by the Thomas
// method the paper names for Eq (2.3), and x^y and ln x by the C library.
// kFlagContract instead evaluates those three pieces in the fixed order of
// operations that the GPU library also follows (partitioned elimination with
// a cyclic-reduction reduced system and fused multiply-adds for the field,
// partitioned elimination for Eq (2.3), ln and exp by written-out series), so
// that whole runs can be compared bit for bit.  Both orders are exact up to
// rounding; the plain path is what pins the other.
constexpr int32_t kFlagContract = 1;
// kFlagLiteralOrder: the electron sub-steps in the order Sec. II.A lists
// them, push, removal, charge assignment, then the collisions, so that a
// particle created by an ionization is first deposited one step after its
// ion (and an attached electron is still deposited in the step it attaches).
// The default deposits after the collisions.
constexpr int32_t kFlagLiteralOrder = 2;

thread_local std::string g_err;

}  // namespace

extern "C" {

// Mirrors the parameters of the discharge problem (see the header comment of
// oracle/__init__.py for the field meanings).  This struct is the oracle's own.
typedef struct orc_channel {
  int32_t kind;     // 0 elastic, 1 excitation, 2 ionization, 3 attachment
  int32_t product;  // ion species that receives the ion of an ionization / attachment
  double threshold_eV;
  const double* sigma_m2;  // n_energy values at E_i = i / inv_de_per_eV
  double target_fraction;  // share of n_gas_m3 that is this channel's target
  double target_mass_amu;  // target mass for the elastic recoil (0: m_gas_amu)
} orc_channel;

// One ion species of the multi-species drift-diffusion model (ion model 4).
typedef struct orc_species {
  int32_t charge;  // +1 or -1
  int32_t n_mu;    // mobility table points
  double m_amu;
  double en_lo_Td, en_hi_Td;  // table abscissae, log-spaced E/N [Td]
  const double* mu_m2_Vs;     // [n_mu]
  double init_fraction;       // initial density / initial electron density
} orc_species;

typedef struct orc_params {
  int32_t precision;  // 0: float particles, 1: double particles
  int32_t ion_model;  // 0/1: drift-diffusion / full fluid with constant mu / nu;
                      // 2/3: the same with the fitted mu(E) / nu(u) of Tables 2 / 3;
                      // 4: drift-diffusion of n_species species with tabulated mu(E/N)
  int32_t n_cells;
  int32_t n_energy;
  int32_t n_channels;
  int32_t sort_every;
  int32_t eedf_every;
  int32_t n_eedf_bins;
  int32_t n_species;  // ion model 4 only
  int32_t flags;      // kFlagContract | kFlagLiteralOrder (see below)
  int64_t n_macro;
  uint64_t seed;
  double n_gas_m3, t_gas_K, m_gas_amu;
  double gap_m;
  double v_amp_V, f_rf_Hz, phase_rad;
  double n_e0_m3, t_e0_eV, load_lo, load_hi;
  double gamma_see, e_sec_eV;
  double m_ion_amu, mu_const, nu_const;
  double dt_s;
  double inv_de_per_eV;
  double eedf_emax_eV;
  double power_W_m2;   // P_0 of Eq 2.9 per electrode area; 0: fixed amplitude
  double power_alpha;  // alpha of Eq 2.9
  const orc_channel* channels;
  const orc_species* species;
} orc_params;

// Auxiliary ion swarm (Sec. II.C): one ion species in a uniform field E_0
// and a Maxwellian background gas, isotropic scattering in the centre of
// mass, no positions (a periodic domain in a uniform field).
typedef struct orc_swarm_params {
  int32_t precision;  // 0: float velocities, 1: double
  int32_t n_fields;   // independent swarms, one per E_0
  int32_t n_energy;   // rate-coefficient table points
  int32_t flags;      // kFlagContract: the series logarithm in the normal deviates
  int64_t n_ions;     // ions per swarm
  int64_t id0;        // stream id of the first ion (a window of a larger swarm)
  uint64_t seed;
  double n_gas_m3, t_gas_K, m_ion_amu, m_gas_amu;
  double t_i0_K;         // initial ion temperature
  double dt_s;
  double inv_de_per_eV;  // table on relative (centre-of-mass) energies i / inv_de_per_eV
  const double* rate_m3_s;  // [n_energy] k = Q_m g at those energies
  const double* e0_V_m;     // [n_fields]
} orc_swarm_params;

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with the round constants of that paper, the key
// bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t y0 = hi1 ^ x1 ^ k0;
    const uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

// A random stream S(tag, id, step): Philox blocks b = 0, 1, 2, ... with
// counter {id, step, b, tag} and key {seed_lo, seed_hi}; the words of each
// block are consumed strictly in order.
struct Stream {
  uint32_t key[2];
  uint32_t ctr[4];
  uint32_t w[4];
  int pos;
  bool narrow = false;  // double uniforms drawn like float ones (decision-locked replay)
  Stream(uint64_t seed, uint32_t tag, uint32_t id, uint32_t step) {
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    ctr[0] = id;
    ctr[1] = step;
    ctr[2] = 0;
    ctr[3] = tag;
    pos = 4;
  }
  uint32_t word() {
    if (pos == 4) {
      philox4x32_10(ctr, key, w);
      ctr[2] += 1;
      pos = 0;
    }
    return w[pos++];
  }
};

// Uniform in [0,1): float from the top 24 bits of one word; double from the
// top 53 bits of two consecutive words (first word high).
inline float uniform_f32(Stream& s) { return (float)(s.word() >> 8) * 0x1p-24f; }
inline double uniform_f64(Stream& s) {
  const uint64_t hi = s.word();
  const uint64_t lo = s.word();
  return (double)(((hi << 32) | lo) >> 11) * 0x1p-53;
}
template <class P> P uniform(Stream& s);
template <> float uniform<float>(Stream& s) { return uniform_f32(s); }
template <> double uniform<double>(Stream& s) {
  return s.narrow ? (double)uniform_f32(s) : uniform_f64(s);
}

enum Tag : uint32_t {
  kTagElectron = 0,
  kTagLoad = 1,
  kTagEmission = 2,
  kTagSwarm = 3,      // swarm steps; + 16 x field index
  kTagSwarmLoad = 4   // swarm initial velocities; + 16 x field index
};

// ---------------------------------------------------------------------------
// Derived constants, computed once in FP64 from the parameters.
// ---------------------------------------------------------------------------
struct Derived {
  int nc, nn;     // cells, nodes
  double L, dz;
  double w;       // superparticle weight per unit electrode area [m^-2], Eq (1.2)
  std::vector<double> dV;     // control length of node j: dz inside, dz/2 at walls
  std::vector<double> scale;  // density per fixed-point count unit at node j
  double kp;        // dz^2 / eps0
  double inv_dz, inv_2dz, hdz_eps;  // 1/dz, 1/(2 dz), dz/(2 eps0)
  double qm_dt;     // (-e/m_e) dt
  // ion fluid
  double M;         // ion mass
  double TN;        // background gas temperature [J]
  double kappa;     // Wannier factor of Eq (2.8): (m_i+m_N)/(5 m_i+3 m_N) m_N
  double dt_2dz, dt_dz;
  double e_M_dt;    // e dt / M
  double dt_2dzM;   // dt / (2 dz M)
  double hdt;       // dt / 2
  double nfloor;    // density below which u = Gamma/n is taken as zero
  // collisions
  double nu_max, Pmax;
  std::vector<double> cum;  // (n_energy x K) cumulative probabilities, FP64
  // electron constants
  double KE;        // m_e/(2e): energy [eV] per (m/s)^2
  double invKE;     // 2e/m_e
  double kdz;       // dt/dz
  double delta;     // 2 m_e / M_gas
  double keedf;     // n_bins / E_max
  std::vector<double> delta_k;  // per channel: 2 m_e / M_target (elastic recoil)
  // ion species of model 4 (one entry, unused, for models 0-3)
  struct Species {
    int Z = 1;           // charge number
    double kappa = 0.0;  // Eq (2.8) factor with this species' mass
    int n = 0;           // mobility table points
    double lo = 0.0, L0 = 0.0, inv_dL = 0.0;  // table start [Td], ln of it, points per ln unit
    std::vector<double> mu;
    double frac = 0.0;   // initial density / initial electron density
  };
  int S = 1;
  std::vector<Species> sp;
  double n_gas = 0.0;
  bool contract = false;  // kFlagContract
  bool literal = false;   // kFlagLiteralOrder
};

bool derive(const orc_params& p, Derived& d) {
  if (p.n_cells < 2 || p.n_energy < 2 || p.n_channels < 0 || p.n_channels > kMaxChannels ||
      p.sort_every < 1 || p.eedf_every < 1 || p.n_eedf_bins < 1 || p.n_macro < 0 ||
      !(p.gap_m > 0) || !(p.dt_s > 0) || !(p.inv_de_per_eV > 0) || !(p.load_hi > p.load_lo) ||
      p.load_lo < 0 || p.load_hi > 1 || (p.ion_model < 0 || p.ion_model > 4) ||
      (p.precision != 0 && p.precision != 1) || (p.n_channels > 0 && !p.channels) ||
      !(p.power_W_m2 >= 0) || !std::isfinite(p.power_W_m2) || !(p.power_alpha >= 0) ||
      !std::isfinite(p.power_alpha) ||
      (p.power_W_m2 > 0 && !(p.f_rf_Hz > 0 && 1.0 / (p.f_rf_Hz * p.dt_s) >= 1.5))) {
    g_err = "invalid parameters";
    return false;
  }
  if (p.flags & ~(kFlagContract | kFlagLiteralOrder)) {
    g_err = "unknown flags";
    return false;
  }
  d.contract = (p.flags & kFlagContract) != 0;
  d.literal = (p.flags & kFlagLiteralOrder) != 0;
  // ion species (model 4) and the products of ionization and attachment
  d.n_gas = p.n_gas_m3;
  if (p.ion_model == 4) {
    if (p.n_species < 1 || p.n_species > 4 || !p.species) {
      g_err = "ion model 4 needs 1 to 4 species";
      return false;
    }
    d.S = p.n_species;
  } else if (p.n_species != 0) {
    g_err = "species are for ion model 4 only";
    return false;
  } else {
    d.S = 1;
  }
  d.sp.assign(d.S, Derived::Species());
  const double mNg = p.m_gas_amu * kAmu;
  if (p.ion_model == 4)
    for (int s = 0; s < d.S; ++s) {
      const orc_species& q = p.species[s];
      if ((q.charge != 1 && q.charge != -1) || q.n_mu < 2 || q.n_mu > 256 || !q.mu_m2_Vs ||
          !(q.m_amu > 0) || !(q.en_lo_Td > 0) || !(q.en_hi_Td > q.en_lo_Td) ||
          !(q.init_fraction >= 0) || !std::isfinite(q.init_fraction)) {
        g_err = "invalid ion species";
        return false;
      }
      Derived::Species& sp = d.sp[s];
      sp.Z = q.charge;
      const double Ms = q.m_amu * kAmu;
      sp.kappa = (Ms + mNg) / (5.0 * Ms + 3.0 * mNg) * mNg;
      sp.n = q.n_mu;
      sp.lo = q.en_lo_Td;
      sp.L0 = std::log(q.en_lo_Td);
      sp.inv_dL = (double)(q.n_mu - 1) / (std::log(q.en_hi_Td) - sp.L0);
      sp.mu.assign(q.mu_m2_Vs, q.mu_m2_Vs + q.n_mu);
      for (double m : sp.mu)
        if (!(m >= 0) || !std::isfinite(m)) {
          g_err = "invalid ion species";
          return false;
        }
      sp.frac = q.init_fraction;
    }
  for (int k = 0; k < p.n_channels; ++k) {
    const orc_channel& c = p.channels[k];
    const bool makes_ion = c.kind == 2 || c.kind == 3;
    if (c.kind < 0 || c.kind > 3 || !(c.target_fraction >= 0) ||
        !std::isfinite(c.target_fraction) || !(c.target_mass_amu >= 0) ||
        (makes_ion && (c.product < 0 || c.product >= d.S)) ||
        (c.kind == 2 && p.ion_model == 4 && d.sp[c.product].Z != 1) ||
        (c.kind == 3 && (p.ion_model != 4 || d.sp[c.product].Z != -1))) {
      g_err = "invalid channel";
      return false;
    }
  }
  d.nc = p.n_cells;
  d.nn = p.n_cells + 1;
  d.L = p.gap_m;
  d.dz = p.gap_m / p.n_cells;
  // Eq (1.2): N_p/sp = n_e0 dV / N_s0 with N_s0 the initial superparticles per
  // cell; per unit electrode area this is n_e0 (hi-lo) L / N_0.
  d.w = p.n_macro > 0 ? p.n_e0_m3 * (p.load_hi - p.load_lo) * p.gap_m / (double)p.n_macro : 0.0;
  d.dV.assign(d.nn, d.dz);
  d.dV[0] = 0.5 * d.dz;
  d.dV[d.nc] = 0.5 * d.dz;
  d.scale.resize(d.nn);
  for (int j = 0; j < d.nn; ++j) d.scale[j] = std::ldexp(d.w, -32) / d.dV[j];
  d.kp = d.dz * d.dz / kEps0;
  d.inv_dz = 1.0 / d.dz;
  d.inv_2dz = 0.5 / d.dz;
  d.hdz_eps = d.dz / (2.0 * kEps0);
  d.qm_dt = (-kE / kMe) * p.dt_s;
  d.M = p.m_ion_amu * kAmu;
  const double mN = p.m_gas_amu * kAmu;
  d.TN = kKb * p.t_gas_K;
  d.kappa = (d.M + mN) / (5.0 * d.M + 3.0 * mN) * mN;
  d.dt_2dz = p.dt_s / (2.0 * d.dz);
  d.dt_dz = p.dt_s / d.dz;
  d.e_M_dt = kE * p.dt_s / d.M;
  d.dt_2dzM = p.dt_s / (2.0 * d.dz * d.M);
  d.hdt = 0.5 * p.dt_s;
  d.nfloor = 1e-10 * p.n_e0_m3;
  // Null-collision tables: nu_k(E_i) = N_g sigma_k(E_i) sqrt(2 e E_i / m_e),
  // nu_max = max_i sum_k nu_k(E_i), P_max = 1 - exp(-nu_max dt); the cumulative
  // probabilities P_max sum_{m<=k} nu_m / nu_max select the channel.
  const int ne = p.n_energy, K = p.n_channels;
  std::vector<double> nu((size_t)ne * K, 0.0);
  d.nu_max = 0.0;
  for (int i = 0; i < ne; ++i) {
    const double Ei = (double)i / p.inv_de_per_eV;
    const double v = std::sqrt(2.0 * kE * Ei / kMe);
    double tot = 0.0;
    for (int k = 0; k < K; ++k) {
      const double s = p.channels[k].sigma_m2[i];
      if (!(s >= 0) || !std::isfinite(s)) {
        g_err = "cross section must be finite and non-negative";
        return false;
      }
      nu[(size_t)i * K + k] = (p.n_gas_m3 * p.channels[k].target_fraction) * s * v;
      tot += nu[(size_t)i * K + k];
    }
    if (tot > d.nu_max) d.nu_max = tot;
  }
  d.Pmax = d.nu_max > 0 ? 1.0 - std::exp(-d.nu_max * p.dt_s) : 0.0;
  d.cum.assign((size_t)ne * K, 0.0);
  for (int i = 0; i < ne; ++i) {
    double acc = 0.0;
    for (int k = 0; k < K; ++k) {
      acc += nu[(size_t)i * K + k];
      d.cum[(size_t)i * K + k] = d.nu_max > 0 ? d.Pmax * acc / d.nu_max : 0.0;
    }
  }
  d.KE = 0.5 * kMe / kE;
  d.invKE = 2.0 * kE / kMe;
  d.kdz = p.dt_s / d.dz;
  d.delta = 2.0 * kMe / (p.m_gas_amu * kAmu);
  d.delta_k.assign(K, 0.0);
  for (int k = 0; k < K; ++k) {
    const double mt = p.channels[k].target_mass_amu > 0 ? p.channels[k].target_mass_amu
                                                         : p.m_gas_amu;
    d.delta_k[k] = 2.0 * kMe / (mt * kAmu);
  }
  d.keedf = (double)p.n_eedf_bins / p.eedf_emax_eV;
  return true;
}

// ---------------------------------------------------------------------------
// Field solve (coupling through Poisson's equation, Sec. II.D).
// rho_j = e (n_i,j - n_e,j);  -phi_{j-1} + 2 phi_j - phi_{j+1} = dz^2 rho_j / eps0
// for the interior nodes, phi_0 = V(t_n) (powered electrode at z = 0) and
// phi_N = 0 (grounded electrode at z = L), solved by the Thomas method (or,
// with kFlagContract, the partitioned elimination with the right-hand side
// carried by fused multiply-adds).  E from centred differences inside and
// from Gauss's law over the half cells at the walls.
// ---------------------------------------------------------------------------
void thomas(int n, const double* a, const double* b, const double* c, const double* dd,
            double* x);
void solve_tridiag(int n, const double* a, const double* b, const double* c, const double* d,
                   double* x);
void solve_tridiag_fma(int n, const double* a, const double* b, const double* c,
                       const double* d, double* x);

void field_solve(const Derived& d, const int64_t* cnt, const double* ni, double V, double* ne_out,
                 double* rho, double* phi, double* E) {
  const int nc = d.nc, nn = d.nn;
  for (int j = 0; j < nn; ++j) {
    ne_out[j] = (double)cnt[j] * d.scale[j];
    rho[j] = kE * (ni[j] - ne_out[j]);
  }
  phi[0] = V;
  phi[nc] = 0.0;
  const int m = nc - 1;
  if (m >= 1) {
    std::vector<double> a(m, -1.0), b(m, 2.0), c(m, -1.0), rhs(m), x(m);
    for (int j = 1; j <= m; ++j) {
      double dj = d.kp * rho[j];
      if (j == 1) dj = dj + phi[0];
      if (j == m) dj = dj + phi[nc];
      rhs[j - 1] = dj;
    }
    if (d.contract)
      solve_tridiag_fma(m, a.data(), b.data(), c.data(), rhs.data(), x.data());
    else
      thomas(m, a.data(), b.data(), c.data(), rhs.data(), x.data());
    for (int j = 1; j <= m; ++j) phi[j] = x[j - 1];
  }
  for (int j = 1; j < nc; ++j) E[j] = (phi[j - 1] - phi[j + 1]) * d.inv_2dz;
  E[0] = (phi[0] - phi[1]) * d.inv_dz - rho[0] * d.hdz_eps;
  E[nc] = (phi[nc - 1] - phi[nc]) * d.inv_dz + rho[nc] * d.hdz_eps;
}

// ---------------------------------------------------------------------------
// Fitted He+ transport in He at atmospheric pressure (Sec. III): the mobility
// as a function of |E| (Table 2) and the momentum-exchange frequency as a
// function of |u| (Table 3), each with its branch change where the table puts
// it (both fits jump slightly there).  The non-integer powers use the
// logarithm and exponential below, written out so that every implementation
// that takes the same steps rounds the same way.
// ---------------------------------------------------------------------------
// ln x, x > 0 finite: x = m 2^k with m in [sqrt(1/2), sqrt(2)); ln m =
// 2 atanh(s), s = (m - 1)/(m + 1), |s| < 0.172, by the odd series to s^21.
double fit_ln(double x) {
  int k = 0;
  double m = std::frexp(x, &k);  // m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m = m * 2.0;
    k = k - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double q = 1.0 / 21.0;
  q = q * z + 1.0 / 19.0;
  q = q * z + 1.0 / 17.0;
  q = q * z + 1.0 / 15.0;
  q = q * z + 1.0 / 13.0;
  q = q * z + 1.0 / 11.0;
  q = q * z + 1.0 / 9.0;
  q = q * z + 1.0 / 7.0;
  q = q * z + 1.0 / 5.0;
  q = q * z + 1.0 / 3.0;
  q = q * z + 1.0;
  return (double)k * 0.69314718055994530942 + (2.0 * s) * q;
}

// exp y, |y| < 700: y = k ln2 + r with k = rint(y / ln2) and ln2 in two parts
// (the first exact in k ln2 for |k| < 2^11), exp r by its Taylor series to
// r^14 (|r| <= 0.347), then the power of two.
double fit_exp(double y) {
  const double k = std::rint(y * 1.44269504088896340736);
  const double r = (y - k * 6.93147180369123816490e-01) - k * 1.90821492927058770002e-10;
  double q = 1.0 / 87178291200.0;
  q = q * r + 1.0 / 6227020800.0;
  q = q * r + 1.0 / 479001600.0;
  q = q * r + 1.0 / 39916800.0;
  q = q * r + 1.0 / 3628800.0;
  q = q * r + 1.0 / 362880.0;
  q = q * r + 1.0 / 40320.0;
  q = q * r + 1.0 / 5040.0;
  q = q * r + 1.0 / 720.0;
  q = q * r + 1.0 / 120.0;
  q = q * r + 1.0 / 24.0;
  q = q * r + 1.0 / 6.0;
  q = q * r + 1.0 / 2.0;
  q = q * r + 1.0;
  q = q * r + 1.0;
  return std::ldexp(q, (int)k);
}

// x^y for x >= 0 (0^y = 0 for the positive exponents used here): the C
// library's pow, or with the contract the series above.
double fit_pow(double x, double y, bool contract) {
  if (!(x > 0.0)) return 0.0;
  return contract ? fit_exp(y * fit_ln(x)) : std::pow(x, y);
}

// Table 2: mu = 1e-3 (1.18 - 0.185 |E|/E0) below E0 = 1.47e6 V/m, 1e-3 0.94
// (E0/|E|)^0.3 from E0 on [m^2/(V s)].
double mobility_fit(double E, bool contract) {
  const double a = std::fabs(E), E0 = 1.47e6;
  if (a < E0) return 1e-3 * (1.18 - 0.185 * (a / E0));
  return 1e-3 * (0.94 * fit_pow(E0 / a, 0.3, contract));
}

// Table 3: nu = 1e10 (2.07 + 0.88 (|u|/u0)^1.89) below u0 = 2e3 m/s, 1e10
// (1.54 + 1.36 |u|/u0) from u0 on [1/s].
double nu_fit(double u, bool contract) {
  const double a = std::fabs(u), u0 = 2e3;
  if (a < u0) return 1e10 * (2.07 + 0.88 * fit_pow(a / u0, 1.89, contract));
  return 1e10 * (1.54 + 1.36 * (a / u0));
}

// ---------------------------------------------------------------------------
// Ion fluid.  Temperature from Eq (2.8), diffusion coefficient from Eq (2.7).
// ---------------------------------------------------------------------------
inline double ion_temperature(const Derived& d, double mu, double E) {
  const double x = mu * std::fabs(E);
  return d.TN + d.kappa * (x * x);
}

// Drift-diffusion (Sec. II.C), explicit: Gamma_j^n from Eq (2.5) with central
// differences, wall fluxes by the field-direction switch (drift only), and the
// continuity update of Eq (2.4) with half cells at the walls.  Returns the wall
// fluxes Gamma_0 and Gamma_N in gw[0], gw[1]; gam receives Gamma^n.
// fit != 0: the mobility of Table 2 at each node's field, else mu_const.
void fluid_dd(const Derived& d, double mu_const, int fit, double* ni, const double* E, double* gam,
              double gw[2]) {
  const int nc = d.nc, nn = d.nn;
  std::vector<double> n0(ni, ni + nn), mu(nn);
  for (int j = 0; j < nn; ++j) mu[j] = fit ? mobility_fit(E[j], d.contract) : mu_const;
  for (int j = 1; j < nc; ++j) {
    const double T = ion_temperature(d, mu[j], E[j]);
    const double D = mu[j] * T / kE;
    gam[j] = mu[j] * n0[j] * E[j] - D * (n0[j + 1] - n0[j - 1]) * d.inv_2dz;
  }
  gam[0] = mu[0] * n0[0] * std::min(E[0], 0.0);
  gam[nc] = mu[nc] * n0[nc] * std::max(E[nc], 0.0);
  for (int j = 1; j < nc; ++j) ni[j] = n0[j] - d.dt_2dz * (gam[j + 1] - gam[j - 1]);
  ni[0] = n0[0] - d.dt_dz * (gam[1] - gam[0]);
  ni[nc] = n0[nc] - d.dt_dz * (gam[nc] - gam[nc - 1]);
  gw[0] = gam[0];
  gw[1] = gam[nc];
}

// Mobility of a species at field E from its table on log-spaced E/N
// (Td = 1e-21 V m^2): linear in ln(E/N) between points, the end values
// outside the table.
double species_mobility(const Derived& d, const Derived::Species& sp, double E) {
  const double x = (std::fabs(E) / d.n_gas) * 1e21;
  if (!(x > sp.lo)) return sp.mu[0];
  const double u = ((d.contract ? fit_ln(x) : std::log(x)) - sp.L0) * sp.inv_dL;
  if (!(u > 0.0)) return sp.mu[0];
  if (!(u < (double)(sp.n - 1))) return sp.mu[sp.n - 1];
  const int k = (int)u;
  const double t = u - (double)k;
  return sp.mu[k] + t * (sp.mu[k + 1] - sp.mu[k]);
}

// Drift-diffusion of one species of charge number Z (Sec. II.C, Eq (2.5)
// with Z): Gamma_j = Z mu_j n_j E_j - D_j (n_{j+1} - n_{j-1}) / (2 dz),
// D_j = mu_j T_j / e, T_j from Eq (2.8) with the species' mass; at the walls
// the drift flux is kept only when it points into the wall; then Eq (2.4).
void fluid_species(const Derived& d, const Derived::Species& sp, double* ni, const double* E,
                   double* gam, double gw[2]) {
  const int nc = d.nc, nn = d.nn;
  std::vector<double> n0(ni, ni + nn), mu(nn);
  for (int j = 0; j < nn; ++j) mu[j] = species_mobility(d, sp, E[j]);
  for (int j = 1; j < nc; ++j) {
    const double x = mu[j] * std::fabs(E[j]);
    const double T = d.TN + sp.kappa * (x * x);
    const double D = mu[j] * T / kE;
    const double zm = (double)sp.Z * mu[j];
    gam[j] = (zm * n0[j]) * E[j] - (D * (n0[j + 1] - n0[j - 1])) * d.inv_2dz;
  }
  gam[0] = std::min((((double)sp.Z * mu[0]) * n0[0]) * E[0], 0.0);
  gam[nc] = std::max((((double)sp.Z * mu[nc]) * n0[nc]) * E[nc], 0.0);
  for (int j = 1; j < nc; ++j) ni[j] = n0[j] - d.dt_2dz * (gam[j + 1] - gam[j - 1]);
  ni[0] = n0[0] - d.dt_dz * (gam[1] - gam[0]);
  ni[nc] = n0[nc] - d.dt_dz * (gam[nc] - gam[nc - 1]);
  gw[0] = gam[0];
  gw[1] = gam[nc];
}

// Thomas algorithm for a general tridiagonal system a_j x_{j-1} + b_j x_j +
// c_j x_{j+1} = d_j, j = 0..n-1 (a_0 and c_{n-1} unused).  One reciprocal of
// the pivot per row.
void thomas(int n, const double* a, const double* b, const double* c, const double* dd,
            double* x) {
  std::vector<double> cp(n), dp(n);
  for (int j = 0; j < n; ++j) {
    double den = b[j];
    if (j > 0) den = b[j] - a[j] * cp[j - 1];
    const double r = 1.0 / den;
    cp[j] = c[j] * r;
    double num = dd[j];
    if (j > 0) num = dd[j] - a[j] * dp[j - 1];
    dp[j] = num * r;
  }
  x[n - 1] = dp[n - 1];
  for (int j = n - 2; j >= 0; --j) x[j] = dp[j] - cp[j] * x[j + 1];
}

// Number of partitions of the partitioned tridiagonal solve for n unknowns:
// the largest P <= 64 with 2 P^2 <= n (about sqrt(n/2)); 0 (plain Thomas)
// below 8 unknowns.
int n_partitions(int n) {
  if (n < 8) return 0;
  int P = 1;
  while (P + 1 <= 64 && 2 * (P + 1) * (P + 1) <= n) ++P;
  return P;
}

// Exact direct solve of a tridiagonal system by partitions (the elimination
// behind the Thomas method, arranged so that the partitions are independent):
// rows [s_p, e_p] with s_p = p n / P.  Inside a partition the interior rows
// are eliminated forward, each expressed as x_i + a''_i x_s + c''_i x_{i+1} =
// d''_i, then backward, x_i = D_i - A_i x_s - C_i x_e (in terms of the
// partition's own first and last unknowns).  The first and last rows of every
// partition then form a tridiagonal system in (x_s0, x_e0, x_s1, x_e1, ...),
// solved by the Thomas method; the interior follows.
void solve_tridiag(int n, const double* a, const double* b, const double* c, const double* d,
                   double* x) {
  const int P = n_partitions(n);
  if (P == 0) {
    thomas(n, a, b, c, d, x);
    return;
  }
  std::vector<double> ap(n), cp(n), dp(n);  // a'', c'', d'' then A, C, D
  std::vector<double> ra(2 * P), rb(2 * P), rc(2 * P), rd(2 * P), rx(2 * P);
  for (int p = 0; p < P; ++p) {
    const int s = (int)((int64_t)p * n / P);
    const int e = (int)((int64_t)(p + 1) * n / P) - 1;
    // forward over the interior rows s+1 .. e-1
    {
      const int i = s + 1;
      const double r = 1.0 / b[i];
      ap[i] = a[i] * r;
      cp[i] = c[i] * r;
      dp[i] = d[i] * r;
    }
    for (int i = s + 2; i <= e - 1; ++i) {
      const double r = 1.0 / (b[i] - a[i] * cp[i - 1]);
      ap[i] = -(a[i] * ap[i - 1]) * r;
      cp[i] = c[i] * r;
      dp[i] = (d[i] - a[i] * dp[i - 1]) * r;
    }
    // backward: x_i = D_i - A_i x_s - C_i x_e (row e-1 keeps its values)
    for (int i = e - 2; i >= s + 1; --i) {
      dp[i] = dp[i] - cp[i] * dp[i + 1];
      ap[i] = ap[i] - cp[i] * ap[i + 1];
      cp[i] = -(cp[i] * cp[i + 1]);
    }
    // the partition's first and last rows, with x_{s+1} and x_{e-1} substituted
    ra[2 * p] = a[s];
    rb[2 * p] = b[s] - c[s] * ap[s + 1];
    rc[2 * p] = -(c[s] * cp[s + 1]);
    rd[2 * p] = d[s] - c[s] * dp[s + 1];
    ra[2 * p + 1] = -(a[e] * ap[e - 1]);
    rb[2 * p + 1] = b[e] - a[e] * cp[e - 1];
    rc[2 * p + 1] = c[e];
    rd[2 * p + 1] = d[e] - a[e] * dp[e - 1];
  }
  thomas(2 * P, ra.data(), rb.data(), rc.data(), rd.data(), rx.data());
  for (int p = 0; p < P; ++p) {
    const int s = (int)((int64_t)p * n / P);
    const int e = (int)((int64_t)(p + 1) * n / P) - 1;
    const double xs = rx[2 * p], xe = rx[2 * p + 1];
    x[s] = xs;
    x[e] = xe;
    for (int i = s + 1; i <= e - 1; ++i) x[i] = (dp[i] - ap[i] * xs) - cp[i] * xe;
  }
}

// The same two solvers with the right-hand side carried by fused
// multiply-adds: every step of a sweep over the right-hand side is one
// rounding.  Forward, d'_i = fma(-(a_i r_i), d'_{i-1}, d_i r_i) with r_i the
// reciprocal pivot; backward, d'_i = fma(-c'_i, d'_{i+1}, d'_i); the reduced
// system and the recovery of the interior likewise.  The pivots and the
// eliminated a'', c'' are computed exactly as above.
void thomas_fma(int n, const double* a, const double* b, const double* c, const double* dd,
                double* x) {
  std::vector<double> cp(n), dp(n);
  for (int j = 0; j < n; ++j) {
    double den = b[j];
    if (j > 0) den = b[j] - a[j] * cp[j - 1];
    const double r = 1.0 / den;
    cp[j] = c[j] * r;
    dp[j] = j > 0 ? std::fma(-(a[j] * r), dp[j - 1], dd[j] * r) : dd[j] * r;
  }
  x[n - 1] = dp[n - 1];
  for (int j = n - 2; j >= 0; --j) x[j] = std::fma(-cp[j], x[j + 1], dp[j]);
}

// Parallel cyclic reduction (Hockney and Jesshope): at stride s = 1, 2, 4,
// ... while s < m, every row i is combined with rows i - s and i + s, which
// moves its couplings to i - 2s and i + 2s; once s >= m each row holds one
// unknown, x_i = d_i (1 / b_i).  Each step uses the previous step's
// coefficients of all rows; a missing neighbour (i - s < 0 or i + s >= m)
// enters with multiplier 0 and value 0.  With alpha_i = -a_i / b_{i-s},
// gamma_i = -c_i / b_{i+s}:  a'_i = alpha_i a_{i-s}, c'_i = gamma_i c_{i+s},
// b'_i = (b_i + alpha_i c_{i-s}) + gamma_i a_{i+s} and
// d'_i = fma(gamma_i, d_{i+s}, fma(alpha_i, d_{i-s}, d_i)).
void pcr_fma(int m, const double* a, const double* b, const double* c, const double* d,
             double* x) {
  std::vector<double> A(a, a + m), B(b, b + m), C(c, c + m), Dv(d, d + m);
  A[0] = 0.0;
  C[m - 1] = 0.0;
  std::vector<double> A2(m), B2(m), C2(m), D2(m);
  for (int s = 1; s < m; s *= 2) {
    for (int i = 0; i < m; ++i) {
      const bool lo = i - s >= 0, hi = i + s < m;
      const double al = lo ? -A[i] / B[i - s] : 0.0;
      const double ga = hi ? -C[i] / B[i + s] : 0.0;
      A2[i] = lo ? al * A[i - s] : 0.0;
      C2[i] = hi ? ga * C[i + s] : 0.0;
      B2[i] = (B[i] + (lo ? al * C[i - s] : 0.0)) + (hi ? ga * A[i + s] : 0.0);
      D2[i] = std::fma(ga, hi ? Dv[i + s] : 0.0, std::fma(al, lo ? Dv[i - s] : 0.0, Dv[i]));
    }
    A.swap(A2);
    B.swap(B2);
    C.swap(C2);
    Dv.swap(D2);
  }
  for (int i = 0; i < m; ++i) x[i] = Dv[i] * (1.0 / B[i]);
}

// Partitions of the field's solver: P = min(64, n/8) (at least 8 rows
// each); below 16 rows the Thomas method.  The reduced system of the
// partitions' first and last rows (2P rows) is solved by parallel cyclic
// reduction, a few steps of independent row updates instead of a chain of
// 2P dependent rows.
int field_partitions(int n) { return n < 16 ? 0 : std::min(64, n / 8); }

void solve_tridiag_fma(int n, const double* a, const double* b, const double* c,
                       const double* d, double* x) {
  const int P = field_partitions(n);
  if (P == 0) {
    thomas_fma(n, a, b, c, d, x);
    return;
  }
  std::vector<double> ap(n), cp(n), dp(n);
  std::vector<double> ra(2 * P), rb(2 * P), rc(2 * P), rd(2 * P), rx(2 * P);
  for (int p = 0; p < P; ++p) {
    const int s = (int)((int64_t)p * n / P);
    const int e = (int)((int64_t)(p + 1) * n / P) - 1;
    {
      const int i = s + 1;
      const double r = 1.0 / b[i];
      ap[i] = a[i] * r;
      cp[i] = c[i] * r;
      dp[i] = d[i] * r;
    }
    for (int i = s + 2; i <= e - 1; ++i) {
      const double r = 1.0 / (b[i] - a[i] * cp[i - 1]);
      ap[i] = -(a[i] * ap[i - 1]) * r;
      cp[i] = c[i] * r;
      dp[i] = std::fma(-(a[i] * r), dp[i - 1], d[i] * r);
    }
    for (int i = e - 2; i >= s + 1; --i) {
      dp[i] = std::fma(-cp[i], dp[i + 1], dp[i]);
      ap[i] = ap[i] - cp[i] * ap[i + 1];
      cp[i] = -(cp[i] * cp[i + 1]);
    }
    ra[2 * p] = a[s];
    rb[2 * p] = b[s] - c[s] * ap[s + 1];
    rc[2 * p] = -(c[s] * cp[s + 1]);
    rd[2 * p] = std::fma(-c[s], dp[s + 1], d[s]);
    ra[2 * p + 1] = -(a[e] * ap[e - 1]);
    rb[2 * p + 1] = b[e] - a[e] * cp[e - 1];
    rc[2 * p + 1] = c[e];
    rd[2 * p + 1] = std::fma(-a[e], dp[e - 1], d[e]);
  }
  pcr_fma(2 * P, ra.data(), rb.data(), rc.data(), rd.data(), rx.data());
  for (int p = 0; p < P; ++p) {
    const int s = (int)((int64_t)p * n / P);
    const int e = (int)((int64_t)(p + 1) * n / P) - 1;
    const double xs = rx[2 * p], xe = rx[2 * p + 1];
    x[s] = xs;
    x[e] = xe;
    for (int i = s + 1; i <= e - 1; ++i) x[i] = std::fma(-cp[i], xe, std::fma(-ap[i], xs, dp[i]));
  }
}

// Full fluid (Sec. II.B): Eq (2.3) for Gamma^{n+1/2} with the lagged friction
// frequency nu^n and semi-implicit advection, solved by the Thomas method;
// Gamma at the wall nodes from the field-direction switch with mu = e/(M nu)
// (Eq (2.6)); then Eq (2.4) with G^n applied by the caller.  gam holds
// Gamma^{n-1/2} on entry and Gamma^{n+1/2} on exit.
// fit != 0: the frequency of Table 3 at each node's lagged u, else nu_const.
void fluid_full(const Derived& d, double nu_const, int fit, double* ni, const double* E,
                double* gam, double gw[2]) {
  const int nc = d.nc, nn = d.nn;
  std::vector<double> n0(ni, ni + nn), g0(gam, gam + nn), u(nn), T(nn), nu(nn), mu(nn);
  for (int j = 0; j < nn; ++j) {
    u[j] = (n0[j] > d.nfloor) ? g0[j] / n0[j] : 0.0;
    nu[j] = fit ? nu_fit(u[j], d.contract) : nu_const;
    mu[j] = kE / (d.M * nu[j]);
    T[j] = ion_temperature(d, mu[j], E[j]);
  }
  const double gl = mu[0] * n0[0] * std::min(E[0], 0.0);
  const double gr = mu[nc] * n0[nc] * std::max(E[nc], 0.0);
  const int m = nc - 1;
  std::vector<double> a(m), b(m), c(m), rhs(m), x(m);
  for (int j = 1; j <= m; ++j) {
    const int r = j - 1;
    a[r] = -d.dt_2dz * u[j - 1];
    b[r] = 1.0 + nu[j] * d.hdt;
    c[r] = d.dt_2dz * u[j + 1];
    rhs[r] = g0[j] * (1.0 - nu[j] * d.hdt) + d.e_M_dt * n0[j] * E[j] -
             d.dt_2dzM * (n0[j + 1] * T[j + 1] - n0[j - 1] * T[j - 1]);
  }
  rhs[0] = rhs[0] - a[0] * gl;
  rhs[m - 1] = rhs[m - 1] - c[m - 1] * gr;
  if (d.contract)
    solve_tridiag(m, a.data(), b.data(), c.data(), rhs.data(), x.data());
  else
    thomas(m, a.data(), b.data(), c.data(), rhs.data(), x.data());
  gam[0] = gl;
  gam[nc] = gr;
  for (int j = 1; j <= m; ++j) gam[j] = x[j - 1];
  for (int j = 1; j < nc; ++j) ni[j] = n0[j] - d.dt_2dz * (gam[j + 1] - gam[j - 1]);
  ni[0] = n0[0] - d.dt_dz * (gam[1] - gam[0]);
  ni[nc] = n0[nc] - d.dt_dz * (gam[nc] - gam[nc - 1]);
  gw[0] = gl;
  gw[1] = gr;
}

// ---------------------------------------------------------------------------
// Electrons (Sec. II.A).
// ---------------------------------------------------------------------------
template <class P>
struct Particle {
  int32_t c;  // cell index; -1 marks a removed particle (a hole until compaction)
  P off;      // position inside the cell, in [0, 1)
  P vx, vy, vz;
  uint32_t id;
};

// Electron-side constants rounded to the particle precision.
template <class P>
struct PConst {
  P Pmax, KE, invKE, inv_dE, kdz, delta, keedf;
  P thr[kMaxChannels];
  P delta_k[kMaxChannels];
  int kind[kMaxChannels];
  int product[kMaxChannels];
  int K, ne, nbins, nc;
  std::vector<P> tab;  // (ne x K) cumulative probabilities rounded to P
  bool narrow = false; // uniforms drawn as floats (the following run of a replay)
};

template <class P>
void make_pconst(const orc_params& p, const Derived& d, PConst<P>& q) {
  q.Pmax = (P)d.Pmax;
  q.KE = (P)d.KE;
  q.invKE = (P)d.invKE;
  q.inv_dE = (P)p.inv_de_per_eV;
  q.kdz = (P)d.kdz;
  q.delta = (P)d.delta;
  q.keedf = (P)d.keedf;
  q.K = p.n_channels;
  q.ne = p.n_energy;
  q.nbins = p.n_eedf_bins;
  q.nc = d.nc;
  for (int k = 0; k < q.K; ++k) {
    q.thr[k] = (P)p.channels[k].threshold_eV;
    q.kind[k] = p.channels[k].kind;
    q.product[k] = p.channels[k].product;
    q.delta_k[k] = (P)d.delta_k[k];
  }
  q.tab.resize(d.cum.size());
  for (size_t i = 0; i < d.cum.size(); ++i) q.tab[i] = (P)d.cum[i];
}

// Leapfrog push with linear (cloud-in-cell) gather, 1D3V: only v_z is
// accelerated.  Ep holds (-e/m_e) dt E_j at the nodes.  Returns 0 when the
// particle stays inside, 1 when it leaves through z = 0, 2 through z = L.
template <class P>
int push(int32_t& c, P& off, P& vz, const P* Ep, int nc, P kdz) {
  const P e0 = Ep[c];
  const P e1 = Ep[c + 1];
  const P t1 = e1 - e0;
  const P g = e0 + off * t1;
  vz = vz + g;
  const P s = off + vz * kdz;
  const P f = std::floor(s);
  if (!(f >= (P)(-c))) return 1;
  if (f >= (P)(nc - c)) return 2;
  int32_t cn = c + (int32_t)f;
  P on = s - f;
  if (on == (P)1) {
    cn = cn + 1;
    on = (P)0;
  }
  c = cn;
  off = on;
  return 0;
}

// Marsaglia (1972): a point on the unit sphere from a uniform point in the
// unit disk, (2a sqrt(1-q), 2b sqrt(1-q), 1-2q) with q = a^2 + b^2.
// Decision-locked replay: the run in float records every decision that
// floating point takes (removal, channel, the accepted try of each disk
// rejection, the number of secondaries, the sort order); the run in double
// draws the same uniforms (Stream::narrow) and takes the recorded decisions
// instead of its own, so that the two runs follow the same particles and
// differ only by the rounding of their arithmetic.  Lock carries one
// particle's decisions of the collision step.
struct Lock {
  bool follow = false;    // take the recorded decisions (else record them)
  int channel = -1;       // -1: no collision
  int tries[2] = {-1, -1};  // accepted try of the 1st / 2nd sphere, -1: none
  int n_sphere = 0;       // spheres drawn so far in this collision
  int flips = 0;          // decisions of the following run that differed
};

template <class P>
void sphere(Stream& s, P n[3], Lock* lk = nullptr) {
  const int idx = lk ? lk->n_sphere++ : 0;
  const int forced = (lk && lk->follow) ? lk->tries[idx] : -2;
  int took = -1;
  for (int t = 0; t < kSphereTries; ++t) {
    const P a = (P)2 * uniform<P>(s) - (P)1;
    const P b = (P)2 * uniform<P>(s) - (P)1;
    const P q = a * a + b * b;
    const bool own = q < (P)1;
    const bool take = forced == -2 ? own : t == forced;
    if (forced != -2 && own != (t == forced) && t <= forced) lk->flips += 1;
    if (take) {
      P h = (P)1 - q;
      if (h < (P)0) h = (P)0;  // a forced try a rounding outside the disk
      const P r = (P)2 * std::sqrt(h);
      n[0] = a * r;
      n[1] = b * r;
      n[2] = (P)1 - (P)2 * q;
      took = t;
      break;
    }
  }
  if (lk && !lk->follow) lk->tries[idx] = took;
  if (took >= 0) return;
  n[0] = (P)0;
  n[1] = (P)0;
  n[2] = (P)1;
}

// Outcome of the collision step for one particle.
template <class P>
struct Mcc {
  int channel = -1;     // -1: no collision (null or not a candidate)
  bool overflow = false;
  bool child = false;
  bool attached = false;
  Particle<P> kid;
};

// Null-collision Monte Carlo (Sec. II.A): one uniform R per particle; R <
// P_max makes it a candidate; the channel is the first k whose interpolated
// cumulative probability exceeds R.  Isotropic scattering for every channel
// ("scattering on a sphere"), elastic recoil loss 2 m_e/M (1 - cos chi),
// excitation loses the threshold, ionization shares the remaining energy
// uniformly between the primary and a new electron created at the same place
// (Sec. II.D).
template <class P>
Mcc<P> collide(Particle<P>& pt, const PConst<P>& q, uint64_t seed, uint32_t step,
               Lock* lk = nullptr) {
  Mcc<P> r;
  Stream st(seed, kTagElectron, pt.id, step);
  st.narrow = q.narrow;
  const P u0 = uniform<P>(st);
  if (!(u0 < q.Pmax)) {
    if (lk && lk->follow && lk->channel >= 0) lk->flips += 1;
    if (!(lk && lk->follow && lk->channel >= 0)) {
      if (lk) lk->channel = -1;
      return r;
    }
  }
  const P v2 = (pt.vx * pt.vx + pt.vy * pt.vy) + pt.vz * pt.vz;
  const P en = q.KE * v2;
  const P s = en * q.inv_dE;
  int i;
  P t;
  if (s >= (P)(q.ne - 1)) {
    i = q.ne - 2;
    t = (P)1;
    r.overflow = true;
  } else {
    i = (int)s;
    t = s - (P)i;
  }
  int ch = -1;
  for (int k = 0; k < q.K; ++k) {
    const P pa = q.tab[(size_t)i * q.K + k];
    const P pb = q.tab[(size_t)(i + 1) * q.K + k];
    const P pk = pa + t * (pb - pa);
    if (u0 < pk) {
      ch = k;
      break;
    }
  }
  if (lk) {
    if (lk->follow) {
      if (ch != lk->channel) lk->flips += 1;
      ch = lk->channel;
    } else {
      lk->channel = ch;
    }
  }
  r.channel = ch;
  if (ch < 0) return r;
  const int kind = q.kind[ch];
  P n[3];
  if (kind == 0) {
    sphere(st, n, lk);
    const P vm = std::sqrt(v2);
    const P cosx = ((pt.vx * n[0] + pt.vy * n[1]) + pt.vz * n[2]) / vm;
    const P fac = (P)1 - q.delta_k[ch] * ((P)1 - cosx);
    const P vn = std::sqrt(v2 * fac);
    pt.vx = vn * n[0];
    pt.vy = vn * n[1];
    pt.vz = vn * n[2];
  } else if (kind == 3) {
    // attachment: the electron is lost to a negative ion at its position
    r.attached = true;
  } else if (kind == 1) {
    sphere(st, n, lk);
    P er = en - q.thr[ch];
    if (er < (P)0) er = (P)0;
    const P vn = std::sqrt(er * q.invKE);
    pt.vx = vn * n[0];
    pt.vy = vn * n[1];
    pt.vz = vn * n[2];
  } else {
    sphere(st, n, lk);
    const P us = uniform<P>(st);
    P er = en - q.thr[ch];
    if (er < (P)0) er = (P)0;
    const P es = us * er;
    const P ep = er - es;
    const P vn = std::sqrt(ep * q.invKE);
    pt.vx = vn * n[0];
    pt.vy = vn * n[1];
    pt.vz = vn * n[2];
    P m2[3];
    sphere(st, m2, lk);
    const P vc = std::sqrt(es * q.invKE);
    r.child = true;
    r.kid.c = pt.c;
    r.kid.off = pt.off;
    r.kid.vx = vc * m2[0];
    r.kid.vy = vc * m2[1];
    r.kid.vz = vc * m2[2];
    r.kid.id = 0;
  }
  return r;
}

// Cloud-in-cell charge assignment in 64-bit fixed point: weight
// W1 = rint(off 2^32) on node c+1 and 2^32 - W1 on node c.
template <class P>
inline void deposit(int32_t c, P off, int64_t* g) {
  const int64_t W1 = (int64_t)std::rint(off * (P)4294967296.0);
  const int64_t W0 = ((int64_t)1 << 32) - W1;
  g[c] += W0;
  g[c + 1] += W1;
}

template <class P>
inline int eedf_bin(const Particle<P>& p, const PConst<P>& q) {
  const P en = q.KE * ((p.vx * p.vx + p.vy * p.vy) + p.vz * p.vz);
  const P x = en * q.keedf;
  return (x < (P)q.nbins) ? (int)x : q.nbins;
}

struct Counters {
  uint64_t coll[kMaxChannels] = {};
  uint64_t absorbed[2] = {};
  uint64_t emitted[2] = {};
  uint64_t created = 0;
  uint64_t overflow = 0;
  uint64_t see_clamped = 0;
  uint64_t pushed = 0;  // particle-steps: live particles pushed
};

// Threads of the particle loop (1: the plain serial loop).
int g_threads = 1;

// The decisions of one step of a replay's recording run (see Lock), per
// array slot where they concern a particle.
struct Trace {
  std::vector<int8_t> out;       // push result: 0 stays, 1 left through z = 0, 2 through z = L
  std::vector<int8_t> chan;      // collision channel, -1 none
  std::vector<int8_t> tries;     // accepted try of the first and second sphere, -1 none
  int64_t see[2] = {0, 0};       // secondaries drawn per side
  std::vector<int8_t> see_keep;  // per secondary (side s at s * 4096 + index): inside the gap
  std::vector<uint32_t> order;   // slots kept by the sort, in their new order
};

// Decisions of a replay's following run that its own arithmetic would have
// taken differently.
struct Flips {
  int64_t removal = 0, mcc = 0, emission = 0, sort = 0;
};

// ---------------------------------------------------------------------------
// One discharge.
// ---------------------------------------------------------------------------
struct Base {
  orc_params p;
  std::vector<orc_channel> ch;
  std::vector<std::vector<double>> sig;
  Derived d;
  int64_t step = 0;
  uint32_t next_id = 0;
  std::vector<int64_t> cnt, ion_src;
  std::vector<double> ni, gam, ne, rho, phi, E;
  std::vector<uint64_t> acc_cnt, eedf;
  std::vector<double> acc_ni;
  uint64_t n_acc = 0;
  Counters ctr;
  // RF drive and absorbed power (Sec. II.D, Eq 2.9)
  int64_t rf_steps = 0;     // steps per RF period, round(1/(f dt)); 0: none
  double amp = 0.0;         // amplitude for the levels after the current one
  double V_cur = 0.0;       // electrode voltage of the current level
  double pw_sum = 0.0;      // the current period's sum of interval powers
  double p_abs = 0.0;       // P_abs of the last completed period
  int64_t rf_periods = 0;
  std::vector<int64_t> last_src;  // ion sources of the last step (fixed point)
  Trace* rec = nullptr;           // replay: record this run's decisions here
  const Trace* follow = nullptr;  // replay: take these decisions instead
  Flips flips;
  bool replay_failed = false;
  int fail_replay(const char* why) {
    g_err = why;
    replay_failed = true;
    return -1;
  }
  virtual ~Base() {}
  virtual int do_step() = 0;
  virtual int64_t count() const = 0;
  virtual void get(int32_t*, void*, void*, void*, void*, uint32_t*) const = 0;
  virtual void get_ep(void*) const = 0;
  virtual void set_particles(int64_t, const int32_t*, const void*, const void*, const void*,
                             const void*, const uint32_t*) = 0;

  // V(t_n) = U sin(2 pi f t_n + phase) at z = 0; this is the sine factor.
  double wave(int64_t n) const {
    const double two_pi_f = 2.0 * kPi * p.f_rf_Hz;
    const double t = (double)n * p.dt_s;
    return std::sin(two_pi_f * t + p.phase_rad);
  }
  void init_drive() {
    if (p.f_rf_Hz > 0) {
      const double r = 1.0 / (p.f_rf_Hz * p.dt_s);
      rf_steps = r < 4.0e18 ? (int64_t)std::llround(r) : 0;
    }
    amp = p.v_amp_V;
    V_cur = amp * wave(0);
  }
  // Ion charge density / e at the nodes: n_i itself for one species, else
  // sum_s Z_s n_s (species in order).  ni and gam hold the species one
  // after another (nn values each).
  std::vector<double> net_of(const std::vector<double>& a) const {
    const int nn = d.nn;
    if (p.ion_model != 4) return std::vector<double>(a.begin(), a.begin() + nn);
    std::vector<double> out(nn);
    for (int j = 0; j < nn; ++j) {
      double v = (double)d.sp[0].Z * a[j];
      for (int q = 1; q < d.S; ++q) v = v + (double)d.sp[q].Z * a[(size_t)q * nn + j];
      out[j] = v;
    }
    return out;
  }
  void field() {
    const std::vector<double> nq = net_of(ni);
    field_solve(d, cnt.data(), nq.data(), V_cur, ne.data(), rho.data(), phi.data(), E.data());
  }

  // After step n (step already advanced to n+1): the power delivered at the
  // driven electrode z = 0 over [t_n, t_n+1] is the mean voltage times the
  // total current density there: conduction e (Gamma_i - Gamma_e), with the
  // ion wall flux gi0 of the step and Gamma_e from the electrons emitted
  // minus absorbed at z = 0 during the step, plus displacement eps0 dE_0/dt.
  // It is added to the period containing t_n+1; a period ends at the levels
  // that are multiples of rf_steps, and its mean is P_abs of Eq 2.9, which
  // rescales the amplitude of the following levels when P_0 > 0.
  void power_step(double gi0, uint64_t abs_before, uint64_t emi_before) {
    const double e0_old = E[0];  // field of level n (solved at the step's start)
    const double v_old = V_cur;
    const double v_new = amp * wave(step);
    const std::vector<double> nq = net_of(ni);
    field_solve(d, cnt.data(), nq.data(), v_new, ne.data(), rho.data(), phi.data(), E.data());
    const double dn =
        (double)(ctr.emitted[0] - emi_before) - (double)(ctr.absorbed[0] - abs_before);
    const double ge = (d.w * dn) / p.dt_s;
    const double jc = kE * (gi0 - ge);
    const double jd = kEps0 * ((E[0] - e0_old) / p.dt_s);
    pw_sum = pw_sum + (0.5 * (v_old + v_new)) * (jc + jd);
    V_cur = v_new;
    if (rf_steps > 0 && step % rf_steps == 0) {
      const double pa = pw_sum / (double)rf_steps;
      p_abs = pa;
      rf_periods += 1;
      if (p.power_W_m2 > 0) amp = amp * (1.0 - p.power_alpha * ((pa - p.power_W_m2) / p.power_W_m2));
      pw_sum = 0.0;
    }
  }
};

template <class P>
struct Discharge : Base {
  PConst<P> q;
  std::vector<Particle<P>> parts;
  std::vector<P> Ep;

  bool init() {
    make_pconst(p, d, q);
    const int nn = d.nn;
    cnt.assign(nn, 0);
    ion_src.assign((size_t)d.S * nn, 0);
    last_src.assign((size_t)d.S * nn, 0);
    ni.assign((size_t)d.S * nn, 0.0);
    gam.assign((size_t)d.S * nn, 0.0);
    ne.assign(nn, 0.0);
    rho.assign(nn, 0.0);
    phi.assign(nn, 0.0);
    E.assign(nn, 0.0);
    Ep.assign(nn, (P)0);
    acc_cnt.assign(nn, 0);
    acc_ni.assign(nn, 0.0);
    eedf.assign((size_t)p.n_eedf_bins + 1, 0);
    load();
    init_drive();
    // Ions start equal to the deposited electron density, so the net charge
    // is exactly zero at t = 0; Gamma^{-1/2} = 0.
    // With several species, species s starts at init_fraction_s times it.
    for (int j = 0; j < nn; ++j) ni[j] = (double)cnt[j] * d.scale[j];
    if (p.ion_model == 4)
      for (int q = d.S - 1; q >= 0; --q)
        for (int j = 0; j < nn; ++j) ni[(size_t)q * nn + j] = d.sp[q].frac * ni[j];
    return true;
  }

  // Initial load (Sec. II.A, Eq (1.1)-(1.2)): uniform positions in
  // [lo L, hi L), isotropic Maxwellian velocities with kT = t_e0 (three normal
  // deviates from two Marsaglia polar pairs), stream (tag 1, id = k, step 0).
  void load() {
    const int64_t N = p.n_macro;
    parts.resize((size_t)N);
    const double vth = std::sqrt(p.t_e0_eV * kE / kMe);
    for (int64_t k = 0; k < N; ++k) {
      Stream st(p.seed, kTagLoad, (uint32_t)k, 0);
      const double u0 = uniform_f64(st);
      const double z = p.gap_m * (p.load_lo + (p.load_hi - p.load_lo) * u0);
      const double s = z / d.dz;
      const double fl = std::floor(s);
      int32_t c = (int32_t)fl;
      P off = (P)(s - fl);
      if (off == (P)1) {
        c = c + 1;
        off = (P)0;
      }
      double g[4];
      for (int pair = 0; pair < 2; ++pair) {
        double a = 0, b = 0, qq = 0;
        for (;;) {
          a = 2.0 * uniform_f64(st) - 1.0;
          b = 2.0 * uniform_f64(st) - 1.0;
          qq = a * a + b * b;
          if (qq < 1.0 && qq > 0.0) break;
        }
        const double f = std::sqrt(-2.0 * std::log(qq) / qq);
        g[2 * pair] = a * f;
        g[2 * pair + 1] = b * f;
      }
      Particle<P>& pt = parts[(size_t)k];
      pt.c = c;
      pt.off = off;
      pt.vx = (P)(vth * g[0]);
      pt.vy = (P)(vth * g[1]);
      pt.vz = (P)(vth * g[2]);
      pt.id = (uint32_t)k;
      deposit<P>(c, off, cnt.data());
    }
    next_id = (uint32_t)N;
    // The load ends with the same stable sort by cell as the periodic one.
    std::stable_sort(parts.begin(), parts.end(),
                     [](const Particle<P>& x, const Particle<P>& y) { return x.c < y.c; });
  }

  // Secondary electrons from the ion wall flux (Sec. II.D): X = gamma F dt / w
  // superparticles per step, int(X) plus one more with probability X - int(X).
  // Emission energy e_sec, cosine law in polar angle, uniform azimuth (disk
  // rejection), placed at a uniformly random fraction of one step's flight.
  void emit(int side, double F, uint32_t n, std::vector<Particle<P>>& out) {
    Stream st(p.seed, kTagEmission, (uint32_t)side, n);
    const double X = ((p.gamma_see * F) * p.dt_s) / d.w;
    const double fl = std::floor(X);
    const double ub = uniform_f64(st);
    int64_t ns = (int64_t)fl + ((ub < X - fl) ? 1 : 0);
    if (rec) rec->see[side] = ns;
    if (follow && follow->see[side] != ns) {
      flips.emission += 1;
      ns = follow->see[side];
    }
    if (ns > kSeeMaxPerSide) {
      ctr.see_clamped += (uint64_t)(ns - kSeeMaxPerSide);
      ns = kSeeMaxPerSide;
    }
    const double v = std::sqrt(p.e_sec_eV * d.invKE);
    for (int64_t s = 0; s < ns; ++s) {
      const double uc = uniform_f64(st);
      const double cth = std::sqrt(uc);
      const double sth = std::sqrt(1.0 - uc);
      double a = 1.0, b = 0.0, qq = 1.0;
      for (int t = 0; t < kSphereTries; ++t) {
        const double ta = 2.0 * uniform_f64(st) - 1.0;
        const double tb = 2.0 * uniform_f64(st) - 1.0;
        const double tq = ta * ta + tb * tb;
        if (tq < 1.0 && tq > 0.0) {
          a = ta;
          b = tb;
          qq = tq;
          break;
        }
      }
      const double cph = (a * a - b * b) / qq;
      const double sph = (2.0 * a * b) / qq;
      const double vz = v * cth;
      const double vp = v * sth;
      const double upp = uniform_f64(st);
      const double flight = (vz * p.dt_s) * upp;
      const double z = side == 0 ? flight : d.L - flight;
      const double sc = z / d.dz;
      const double fc = std::floor(sc);
      ctr.emitted[side] += 1;
      bool inside = fc > -2147483648.0 && fc < 2147483647.0;  // a cell index at all
      int32_t c = 0;
      P off = (P)0;
      if (inside) {
        c = (int32_t)fc;
        off = (P)(sc - fc);
        if (off == (P)1) {
          c = c + 1;
          off = (P)0;
        }
        inside = c >= 0 && c < d.nc;
      }
      const size_t slot = (size_t)side * (size_t)kSeeMaxPerSide + (size_t)s;
      if (rec) rec->see_keep[slot] = inside ? 1 : 0;
      if (follow && (follow->see_keep[slot] != 0) != inside) {
        flips.emission += 1;
        inside = !inside;
        if (inside) {  // the recorded run kept it: place it at the wall
          c = side == 0 ? 0 : d.nc - 1;
          off = side == 0 ? (P)0 : std::nextafter((P)1, (P)0);
        }
      }
      if (!inside) {
        ctr.absorbed[side] += 1;
        continue;
      }
      Particle<P> e;
      e.c = c;
      e.off = off;
      e.vx = (P)(vp * cph);
      e.vy = (P)(vp * sph);
      e.vz = (P)(side == 0 ? vz : -vz);
      e.id = 0;
      out.push_back(e);
    }
  }

  // What one thread accumulates over its share of the particle array: the
  // deposit and ion-source grids are integers and the counters are counts,
  // so the sums over threads do not depend on how the array is split, and the
  // children are concatenated in thread order, which is array order.
  struct Local {
    std::vector<int64_t> nxt, src;
    std::vector<uint64_t> eedf;
    std::vector<Particle<P>> kids;
    Counters ctr;
    int64_t flips_removal = 0, flips_mcc = 0;
  };

  // Sec. II.A for the slots [k0, k1) of the particle array in order: push,
  // removal, collision and deposit of each live particle (by default the
  // deposit follows the collision, so that an ionization's new electron is
  // assigned in the same step as its ion; kFlagLiteralOrder assigns the
  // charge before the collisions, as the section lists the sub-steps).
  void electrons(size_t k0, size_t k1, uint32_t n, bool sample, Local& o) {
    const bool lit = d.literal;
    for (size_t k = k0; k < k1; ++k) {
      Particle<P>& pt = parts[k];
      if (pt.c < 0) continue;
      o.ctr.pushed += 1;
      int out = push<P>(pt.c, pt.off, pt.vz, Ep.data(), d.nc, q.kdz);
      if (rec) rec->out[k] = (int8_t)out;
      if (follow && follow->out[k] != out) {
        o.flips_removal += 1;
        if (follow->out[k] == 0) {  // the recorded run kept it: place it at the wall
          pt.c = out == 1 ? 0 : d.nc - 1;
          pt.off = out == 1 ? (P)0 : std::nextafter((P)1, (P)0);
        }
        out = follow->out[k];
      }
      if (out != 0) {
        o.ctr.absorbed[out - 1] += 1;
        pt.c = -1;
        continue;
      }
      if (lit) deposit<P>(pt.c, pt.off, o.nxt.data());
      Lock lk;
      Lock* lkp = nullptr;
      if (rec || follow) {
        lkp = &lk;
        if (follow) {
          lk.follow = true;
          lk.channel = follow->chan[k];
          lk.tries[0] = follow->tries[2 * k];
          lk.tries[1] = follow->tries[2 * k + 1];
        }
      }
      Mcc<P> r = collide<P>(pt, q, p.seed, n, lkp);
      if (rec) {
        rec->chan[k] = (int8_t)lk.channel;
        rec->tries[2 * k] = (int8_t)lk.tries[0];
        rec->tries[2 * k + 1] = (int8_t)lk.tries[1];
      }
      if (follow) o.flips_mcc += lk.flips;
      if (r.overflow) o.ctr.overflow += 1;
      if (r.channel >= 0) o.ctr.coll[r.channel] += 1;
      if (r.attached) {  // the negative ion takes the electron's place and charge
        deposit<P>(pt.c, pt.off, &o.src[(size_t)q.product[r.channel] * d.nn]);
        pt.c = -1;
        continue;
      }
      if (!lit) deposit<P>(pt.c, pt.off, o.nxt.data());
      if (sample) o.eedf[eedf_bin(pt, q)] += 1;
      if (r.child) {
        if (!lit) deposit<P>(r.kid.c, r.kid.off, o.nxt.data());
        deposit<P>(r.kid.c, r.kid.off, &o.src[(size_t)q.product[r.channel] * d.nn]);
        if (sample) o.eedf[eedf_bin(r.kid, q)] += 1;
        o.ctr.created += 1;
        o.kids.push_back(r.kid);
      }
    }
  }

  // The canonical step n (see DESIGN notes in the repository):
  //  1. field from cnt^n, n_i^n and V(t_n);  2. ion fluid with E^n;
  //  3. every particle in array order: push, removal, collision, deposit
  //     (children deposited and their ions recorded at the parent position);
  //  4. secondary emission from the step-2 wall fluxes;  5. append children,
  //  then left then right secondaries, with consecutive ids;  6. ion sources,
  //  run accumulators;  7. every sort_every steps drop holes and sort stably
  //  by cell.
  int do_step() override {
    const uint32_t n = (uint32_t)step;
    const uint64_t abs_before = ctr.absorbed[0], emi_before = ctr.emitted[0];
    field();
    for (int j = 0; j < d.nn; ++j) Ep[j] = (P)(d.qm_dt * E[j]);
    double gw[2];
    double see_flux[2];  // positive-ion flux into each wall (emission)
    if (p.ion_model == 0 || p.ion_model == 2)
      fluid_dd(d, p.mu_const, p.ion_model == 2, ni.data(), E.data(), gam.data(), gw);
    else if (p.ion_model == 1 || p.ion_model == 3)
      fluid_full(d, p.nu_const, p.ion_model == 3, ni.data(), E.data(), gam.data(), gw);
    if (p.ion_model != 4) {
      see_flux[0] = std::max(-gw[0], 0.0);
      see_flux[1] = std::max(gw[1], 0.0);
    } else {
      // every species in order; gw is the net charge flux sum_s Z_s Gamma_s
      gw[0] = gw[1] = 0.0;
      see_flux[0] = see_flux[1] = 0.0;
      for (int q = 0; q < d.S; ++q) {
        double g2[2];
        fluid_species(d, d.sp[q], &ni[(size_t)q * d.nn], E.data(), &gam[(size_t)q * d.nn], g2);
        gw[0] = gw[0] + (double)d.sp[q].Z * g2[0];
        gw[1] = gw[1] + (double)d.sp[q].Z * g2[1];
        if (d.sp[q].Z > 0) {
          see_flux[0] = see_flux[0] + std::max(-g2[0], 0.0);
          see_flux[1] = see_flux[1] + std::max(g2[1], 0.0);
        }
      }
    }
    const bool sample = ((step + 1) % p.eedf_every) == 0;
    const size_t N = parts.size();
    if (rec) {
      rec->out.assign(N, 0);
      rec->chan.assign(N, -1);
      rec->tries.assign(2 * N, -1);
      rec->see_keep.assign(2 * (size_t)kSeeMaxPerSide, 0);
    }
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(g_threads, (int64_t)(N / 4096 + 1)));
    std::vector<Local> loc(T);
    for (Local& o : loc) {
      o.nxt.assign(d.nn, 0);
      o.src.assign((size_t)d.S * d.nn, 0);
      o.eedf.assign((size_t)p.n_eedf_bins + 1, 0);
    }
#pragma omp parallel for num_threads(T) schedule(static, 1)
    for (int t = 0; t < T; ++t)
      electrons(N * (size_t)t / (size_t)T, N * (size_t)(t + 1) / (size_t)T, n, sample, loc[t]);
    std::vector<int64_t> nxt(d.nn, 0);
    std::vector<Particle<P>> kids;
    for (const Local& o : loc) {
      for (int j = 0; j < d.nn; ++j) nxt[j] += o.nxt[j];
      for (size_t j = 0; j < ion_src.size(); ++j) ion_src[j] += o.src[j];
      for (size_t b = 0; b < eedf.size(); ++b) eedf[b] += o.eedf[b];
      kids.insert(kids.end(), o.kids.begin(), o.kids.end());
      for (int k = 0; k < kMaxChannels; ++k) ctr.coll[k] += o.ctr.coll[k];
      for (int s = 0; s < 2; ++s) ctr.absorbed[s] += o.ctr.absorbed[s];
      ctr.created += o.ctr.created;
      ctr.overflow += o.ctr.overflow;
      ctr.pushed += o.ctr.pushed;
      flips.removal += o.flips_removal;
      flips.mcc += o.flips_mcc;
    }
    std::vector<Particle<P>> see[2];
    emit(0, see_flux[0], n, see[0]);
    emit(1, see_flux[1], n, see[1]);
    for (int s = 0; s < 2; ++s)
      for (auto& e : see[s]) deposit<P>(e.c, e.off, nxt.data());
    for (auto& e : kids) {
      e.id = next_id++;
      parts.push_back(e);
    }
    for (int s = 0; s < 2; ++s)
      for (auto& e : see[s]) {
        e.id = next_id++;
        parts.push_back(e);
      }
    cnt.swap(nxt);
    for (int q2 = 0; q2 < d.S; ++q2)
      for (int j = 0; j < d.nn; ++j) {
        const size_t k = (size_t)q2 * d.nn + j;
        ni[k] = ni[k] + (double)ion_src[k] * d.scale[j];
        last_src[k] = ion_src[k];
        ion_src[k] = 0;
      }
    const std::vector<double> nq = net_of(ni);
    for (int j = 0; j < d.nn; ++j) {
      acc_cnt[j] += (uint64_t)cnt[j];
      acc_ni[j] += nq[j];
    }
    n_acc += 1;
    step += 1;
    if (step % p.sort_every == 0) {
      // drop the holes, then a stable sort by cell: the slots kept, in
      // their new order (a replay's following run takes the recorded one)
      std::vector<uint32_t> order;
      if (follow) {
        order = follow->order;
        for (uint32_t k : order)
          if (parts[k].c < 0) return fail_replay("replay order names a hole");
      } else {
        order.reserve(parts.size());
        for (size_t k = 0; k < parts.size(); ++k)
          if (parts[k].c >= 0) order.push_back((uint32_t)k);
        std::stable_sort(order.begin(), order.end(),
                         [&](uint32_t x, uint32_t y) { return parts[x].c < parts[y].c; });
      }
      if (rec) rec->order = order;
      if (follow)
        for (size_t i = 1; i < order.size(); ++i)
          if (parts[order[i]].c < parts[order[i - 1]].c) flips.sort += 1;
      std::vector<Particle<P>> live;
      live.reserve(order.size());
      for (uint32_t k : order) live.push_back(parts[k]);
      parts.swap(live);
    }
    power_step(gw[0], abs_before, emi_before);
    return 0;
  }

  int64_t count() const override { return (int64_t)parts.size(); }
  void get(int32_t* c, void* off, void* vx, void* vy, void* vz, uint32_t* id) const override {
    for (size_t k = 0; k < parts.size(); ++k) {
      const Particle<P>& e = parts[k];
      if (c) c[k] = e.c;
      if (off) ((P*)off)[k] = e.off;
      if (vx) ((P*)vx)[k] = e.vx;
      if (vy) ((P*)vy)[k] = e.vy;
      if (vz) ((P*)vz)[k] = e.vz;
      if (id) id[k] = e.id;
    }
  }
  void get_ep(void* out) const override {
    std::vector<double> ne2(d.nn), rho2(d.nn), phi2(d.nn), E2(d.nn);
    const std::vector<double> nq = net_of(ni);
    field_solve(d, cnt.data(), nq.data(), V_cur, ne2.data(), rho2.data(), phi2.data(),
                E2.data());
    for (int j = 0; j < d.nn; ++j) ((P*)out)[j] = (P)(d.qm_dt * E2[j]);
  }
  void set_particles(int64_t n, const int32_t* c, const void* off, const void* vx, const void* vy,
                     const void* vz, const uint32_t* id) override {
    parts.resize((size_t)n);
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t k = 0; k < n; ++k) {
      Particle<P>& e = parts[(size_t)k];
      e.c = c[k];
      e.off = ((const P*)off)[k];
      e.vx = ((const P*)vx)[k];
      e.vy = ((const P*)vy)[k];
      e.vz = ((const P*)vz)[k];
      e.id = id[k];
      if (e.c >= 0) deposit<P>(e.c, e.off, cnt.data());
    }
  }
};

// Decision-locked replay of one discharge in float and in double (see
// Lock): the float run records, the double run follows with the same
// uniforms, so that the difference of their profiles is the rounding error
// of the float particle arithmetic alone.
struct Replay {
  Base* f = nullptr;
  Base* g = nullptr;
  Trace tr;
  ~Replay() {
    delete f;
    delete g;
  }
  // Give the double run the float run's state (particles converted exactly,
  // grids, sums and counters copied), so that the next step measures the
  // rounding of one step alone.
  void sync() {
    auto* F = static_cast<Discharge<float>*>(f);
    auto* G = static_cast<Discharge<double>*>(g);
    G->parts.resize(F->parts.size());
    for (size_t k = 0; k < F->parts.size(); ++k) {
      const Particle<float>& a = F->parts[k];
      Particle<double>& b = G->parts[k];
      b.c = a.c;
      b.off = a.off;
      b.vx = a.vx;
      b.vy = a.vy;
      b.vz = a.vz;
      b.id = a.id;
    }
    G->cnt = F->cnt;
    G->ion_src = F->ion_src;
    G->ni = F->ni;
    G->gam = F->gam;
    G->ne = F->ne;
    G->rho = F->rho;
    G->phi = F->phi;
    G->E = F->E;
    G->acc_cnt = F->acc_cnt;
    G->acc_ni = F->acc_ni;
    G->eedf = F->eedf;
    G->n_acc = F->n_acc;
    G->ctr = F->ctr;
    G->step = F->step;
    G->next_id = F->next_id;
    G->amp = F->amp;
    G->V_cur = F->V_cur;
    G->pw_sum = F->pw_sum;
    G->p_abs = F->p_abs;
    G->rf_periods = F->rf_periods;
  }
};

Base* make(const orc_params* pp);

Replay* make_replay(const orc_params* pp) {
  if (!pp) return nullptr;
  orc_params a = *pp, b = *pp;
  a.precision = 0;
  b.precision = 1;
  Replay* r = new Replay();
  r->f = make(&a);
  r->g = r->f ? make(&b) : nullptr;
  if (!r->g) {
    delete r;
    return nullptr;
  }
  auto* F = static_cast<Discharge<float>*>(r->f);
  auto* G = static_cast<Discharge<double>*>(r->g);
  G->q.narrow = true;
  // the load sorted each run by its own cells; take the float run's order
  std::vector<size_t> at(G->parts.size());
  for (size_t k = 0; k < G->parts.size(); ++k) at[G->parts[k].id] = k;
  std::vector<Particle<double>> v;
  v.reserve(G->parts.size());
  for (const auto& e : F->parts) v.push_back(G->parts[at[e.id]]);
  G->parts.swap(v);
  r->f->rec = &r->tr;
  r->g->follow = &r->tr;
  return r;
}

Base* make(const orc_params* pp) {
  if (!pp) {
    g_err = "null params";
    return nullptr;
  }
  Base* b = nullptr;
  if (pp->precision == 0)
    b = new Discharge<float>();
  else
    b = new Discharge<double>();
  b->p = *pp;
  // keep private copies of the cross sections
  b->sig.resize(pp->n_channels > 0 ? pp->n_channels : 0);
  b->ch.resize(b->sig.size());
  for (size_t k = 0; k < b->sig.size(); ++k) {
    if (!pp->channels || !pp->channels[k].sigma_m2 || pp->n_energy < 2) {
      g_err = "missing cross section";
      delete b;
      return nullptr;
    }
    b->sig[k].assign(pp->channels[k].sigma_m2, pp->channels[k].sigma_m2 + pp->n_energy);
    b->ch[k] = pp->channels[k];
    b->ch[k].sigma_m2 = b->sig[k].data();
  }
  b->p.channels = b->ch.empty() ? nullptr : b->ch.data();
  if (!derive(b->p, b->d)) {
    delete b;
    return nullptr;
  }
  bool ok = (pp->precision == 0) ? static_cast<Discharge<float>*>(b)->init()
                                 : static_cast<Discharge<double>*>(b)->init();
  if (!ok) {
    delete b;
    return nullptr;
  }
  return b;
}


// ---------------------------------------------------------------------------
// Auxiliary ion Monte Carlo (Sec. II.C): the ions of one species under a
// prescribed uniform field E_0, colliding with a background gas of
// temperature T_N by the null-collision method with sampled targets, reach a
// stationary drift u; the mobility is u / E_0 and Eq (2.6) gives the
// momentum-exchange frequency.  The domain is periodic and the field
// uniform, so positions never enter.  Isotropic scattering in the centre of
// mass with the cross section Q_m = Q_i + 2 Q_b (Sec. III); the caller gives
// the rate coefficient k = Q_m g tabulated on the relative energy
// M_r g^2 / (2e).
// ---------------------------------------------------------------------------

// Two standard normal deviates by Marsaglia's polar method (FP64 uniforms,
// the logarithm above); (0, 0) if no point falls in the disk in
// kSphereTries tries.
void normal_pair(Stream& st, bool contract, double& g0, double& g1) {
  for (int t = 0; t < kSphereTries; ++t) {
    const double a = 2.0 * uniform_f64(st) - 1.0;
    const double b = 2.0 * uniform_f64(st) - 1.0;
    const double q = a * a + b * b;
    if (q < 1.0 && q > 0.0) {
      const double f = std::sqrt((-2.0 * (contract ? fit_ln(q) : std::log(q))) / q);
      g0 = a * f;
      g1 = b * f;
      return;
    }
  }
  g0 = 0.0;
  g1 = 0.0;
}

// Three Cartesian components of a Maxwellian velocity of thermal speed vth
// (two polar pairs, the fourth deviate unused), rounded to P.
template <class P>
void maxwellian(Stream& st, bool contract, double vth, P v[3]) {
  double g[4];
  normal_pair(st, contract, g[0], g[1]);
  normal_pair(st, contract, g[2], g[3]);
  for (int k = 0; k < 3; ++k) v[k] = (P)(vth * g[k]);
}

struct SwarmBase {
  orc_swarm_params p;
  std::vector<double> rate, e0;
  int64_t step = 0;
  std::vector<uint64_t> coll, over;
  std::vector<int64_t> n_acc;  // accumulated steps (the same for every field)
  virtual ~SwarmBase() {}
  virtual void run(int64_t n, int accumulate) = 0;
  virtual void get(int f, void* vx, void* vy, void* vz, double* avz, double* av2) const = 0;
  virtual double sum_vz(int f) const = 0;
  virtual double sum_v2(int f) const = 0;
  bool contract() const { return (p.flags & kFlagContract) != 0; }
};

template <class P>
struct Swarm : SwarmBase {
  double M = 0, MN = 0, vth_n = 0, vth_i0 = 0, Pmax64 = 0, nu_max = 0;
  P Pmax = 0, KEr = 0, inv_dE = 0, m1 = 0, m2 = 0;
  std::vector<P> a;    // [n_fields] velocity gain per step e E_0 dt / M
  std::vector<P> tab;  // [n_energy] Pmax nu(eps_i) / nu_max
  std::vector<P> vx, vy, vz;           // [n_fields * n_ions]
  std::vector<double> avz, av2;        // per-ion sums of v_z and |v|^2 over accumulated steps

  bool init() {
    const int ne = p.n_energy;
    M = p.m_ion_amu * kAmu;
    MN = p.m_gas_amu * kAmu;
    const double Mr = (M * MN) / (M + MN);
    vth_n = std::sqrt(kKb * p.t_gas_K / MN);
    vth_i0 = std::sqrt(kKb * p.t_i0_K / M);
    std::vector<double> nu(ne);
    nu_max = 0.0;
    for (int i = 0; i < ne; ++i) {
      nu[i] = p.n_gas_m3 * rate[i];
      if (nu[i] > nu_max) nu_max = nu[i];
    }
    Pmax64 = 1.0 - std::exp(-nu_max * p.dt_s);
    tab.resize(ne);
    for (int i = 0; i < ne; ++i) tab[i] = (P)(nu_max > 0 ? Pmax64 * (nu[i] / nu_max) : 0.0);
    Pmax = (P)Pmax64;
    KEr = (P)(Mr / (2.0 * kE));
    inv_dE = (P)p.inv_de_per_eV;
    m1 = (P)(M / (M + MN));
    m2 = (P)(MN / (M + MN));
    a.resize(p.n_fields);
    for (int f = 0; f < p.n_fields; ++f) a[f] = (P)(((kE * e0[f]) * p.dt_s) / M);
    const size_t n = (size_t)p.n_fields * (size_t)p.n_ions;
    vx.resize(n);
    vy.resize(n);
    vz.resize(n);
    avz.assign(n, 0.0);
    av2.assign(n, 0.0);
    coll.assign(p.n_fields, 0);
    over.assign(p.n_fields, 0);
    n_acc.assign(p.n_fields, 0);
    // initial Maxwellian at T_i0: stream (kTagSwarmLoad + 16 f, id = ion, step 0)
    for (int f = 0; f < p.n_fields; ++f)
      for (int64_t i = 0; i < p.n_ions; ++i) {
        Stream st(p.seed, kTagSwarmLoad + 16u * (uint32_t)f, (uint32_t)(p.id0 + i), 0);
        P v[3];
        maxwellian<P>(st, contract(), vth_i0, v);
        const size_t k = (size_t)f * (size_t)p.n_ions + (size_t)i;
        vx[k] = v[0];
        vy[k] = v[1];
        vz[k] = v[2];
      }
    return true;
  }

  // One step of one ion: acceleration by the field, then the null-collision
  // test u0 < P_max; for a candidate a gas atom's velocity is drawn from the
  // Maxwellian at T_N, and the collision is real when u0 falls below
  // P_max nu(eps)/nu_max at the pair's relative energy eps = M_r g^2/(2e)
  // (linear interpolation in the table, the last interval beyond its end).
  // A real collision turns the relative velocity to a uniformly random
  // direction of the same length, keeping the centre-of-mass velocity.
  void ion_step(int f, size_t k, uint32_t id) {
    Stream st(p.seed, kTagSwarm + 16u * (uint32_t)f, id, (uint32_t)step);
    vz[k] = vz[k] + a[f];
    const P u0 = uniform<P>(st);
    if (u0 < Pmax) {
      P t3[3];
      maxwellian<P>(st, contract(), vth_n, t3);
      const P gx = vx[k] - t3[0], gy = vy[k] - t3[1], gz = vz[k] - t3[2];
      const P g2 = (gx * gx + gy * gy) + gz * gz;
      const P eps = KEr * g2;
      const P s = eps * inv_dE;
      int i;
      P t;
      if (!(s < (P)(p.n_energy - 1))) {  // beyond the table (or not a number)
        i = p.n_energy - 2;
        t = (P)1;
        over[f] += 1;
      } else {
        i = (int)s;
        t = s - (P)i;
      }
      const P pc = tab[i] + t * (tab[i + 1] - tab[i]);
      if (u0 < pc) {
        P n[3];
        sphere<P>(st, n);
        const P gm = std::sqrt(g2);
        const P r = m2 * gm;
        vx[k] = (m1 * vx[k] + m2 * t3[0]) + r * n[0];
        vy[k] = (m1 * vy[k] + m2 * t3[1]) + r * n[1];
        vz[k] = (m1 * vz[k] + m2 * t3[2]) + r * n[2];
        coll[f] += 1;
      }
    }
  }

  void run(int64_t n, int accumulate) override {
    for (int64_t s = 0; s < n; ++s) {
      for (int f = 0; f < p.n_fields; ++f) {
        for (int64_t i = 0; i < p.n_ions; ++i) {
          const size_t k = (size_t)f * (size_t)p.n_ions + (size_t)i;
          ion_step(f, k, (uint32_t)(p.id0 + i));
          if (accumulate) {
            const double x = (double)vx[k], y = (double)vy[k], z = (double)vz[k];
            avz[k] = avz[k] + z;
            av2[k] = av2[k] + ((x * x + y * y) + z * z);
          }
        }
        if (accumulate) n_acc[f] += 1;
      }
      step += 1;
    }
  }

  void get(int f, void* ox, void* oy, void* oz, double* oa, double* ob) const override {
    for (int64_t i = 0; i < p.n_ions; ++i) {
      const size_t k = (size_t)f * (size_t)p.n_ions + (size_t)i;
      if (ox) ((P*)ox)[i] = vx[k];
      if (oy) ((P*)oy)[i] = vy[k];
      if (oz) ((P*)oz)[i] = vz[k];
      if (oa) oa[i] = avz[k];
      if (ob) ob[i] = av2[k];
    }
  }
  double sum_vz(int f) const override {
    double s = 0.0;
    for (int64_t i = 0; i < p.n_ions; ++i) s += avz[(size_t)f * (size_t)p.n_ions + (size_t)i];
    return s;
  }
  double sum_v2(int f) const override {
    double s = 0.0;
    for (int64_t i = 0; i < p.n_ions; ++i) s += av2[(size_t)f * (size_t)p.n_ions + (size_t)i];
    return s;
  }
};

SwarmBase* make_swarm(const orc_swarm_params* pp) {
  if (!pp || pp->n_fields < 1 || pp->n_energy < 2 || pp->n_ions < 1 || !pp->rate_m3_s ||
      !pp->e0_V_m || !(pp->dt_s > 0) || !(pp->inv_de_per_eV > 0) || !(pp->m_ion_amu > 0) ||
      !(pp->m_gas_amu > 0) || !(pp->n_gas_m3 >= 0) || !(pp->t_gas_K >= 0) || !(pp->t_i0_K >= 0) ||
      pp->id0 < 0 || pp->id0 + pp->n_ions > ((int64_t)1 << 32) ||
      (pp->flags & ~kFlagContract) != 0 ||
      (pp->precision != 0 && pp->precision != 1)) {
    g_err = "invalid swarm parameters";
    return nullptr;
  }
  for (int i = 0; i < pp->n_energy; ++i)
    if (!(pp->rate_m3_s[i] >= 0) || !std::isfinite(pp->rate_m3_s[i])) {
      g_err = "rate coefficients must be finite and non-negative";
      return nullptr;
    }
  SwarmBase* b = pp->precision == 0 ? (SwarmBase*)new Swarm<float>() : (SwarmBase*)new Swarm<double>();
  b->p = *pp;
  b->rate.assign(pp->rate_m3_s, pp->rate_m3_s + pp->n_energy);
  b->e0.assign(pp->e0_V_m, pp->e0_V_m + pp->n_fields);
  b->p.rate_m3_s = b->rate.data();
  b->p.e0_V_m = b->e0.data();
  const bool ok = pp->precision == 0 ? static_cast<Swarm<float>*>(b)->init()
                                     : static_cast<Swarm<double>*>(b)->init();
  if (!ok) {
    delete b;
    return nullptr;
  }
  return b;
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface for the Python test harness.
// ---------------------------------------------------------------------------
extern "C" {

const char* orc_last_error(void) { return g_err.c_str(); }

void* orc_create(const orc_params* p) { return make(p); }
void orc_free(void* h) { delete static_cast<Base*>(h); }

int orc_step(void* h, int64_t n) {
  Base* b = static_cast<Base*>(h);
  if (b->rec || b->follow) {
    g_err = "a replay's runs advance through orc_replay_step";
    return -1;
  }
  for (int64_t i = 0; i < n; ++i)
    if (b->do_step() != 0) return -1;
  return 0;
}

void orc_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int orc_get_threads(void) { return g_threads; }

void orc_get_ion_sources(void* h, int64_t* out) {
  const Base* b = static_cast<Base*>(h);
  std::copy(b->last_src.begin(), b->last_src.end(), out);
}

void* orc_replay_create(const orc_params* p) { return make_replay(p); }
void orc_replay_free(void* r) { delete static_cast<Replay*>(r); }
// which = 0: the float run, 1: the double run (owned by the replay)
void* orc_replay_run(void* r, int which) {
  Replay* x = static_cast<Replay*>(r);
  return which == 0 ? (void*)x->f : (void*)x->g;
}
int orc_replay_step(void* r, int64_t n) {
  Replay* x = static_cast<Replay*>(r);
  for (int64_t i = 0; i < n; ++i) {
    if (x->f->do_step() != 0 || x->g->do_step() != 0) return -1;
    if (x->g->replay_failed) return -1;
  }
  return 0;
}
void orc_replay_sync(void* r) { static_cast<Replay*>(r)->sync(); }
// decisions the double run's own arithmetic took differently
void orc_replay_flips(void* r, int64_t* out) {
  const Flips& f = static_cast<Replay*>(r)->g->flips;
  out[0] = f.removal;
  out[1] = f.mcc;
  out[2] = f.emission;
  out[3] = f.sort;
}

int64_t orc_step_index(void* h) { return static_cast<Base*>(h)->step; }
int64_t orc_num_particles(void* h) { return static_cast<Base*>(h)->count(); }
uint32_t orc_next_id(void* h) { return static_cast<Base*>(h)->next_id; }

void orc_get_particles(void* h, int32_t* c, void* off, void* vx, void* vy, void* vz, uint32_t* id) {
  static_cast<Base*>(h)->get(c, off, vx, vy, vz, id);
}

// Replace the particle population (testing hook): cnt is re-deposited from
// the given particles; ion fields are left untouched.
void orc_set_particles(void* h, int64_t n, const int32_t* c, const void* off, const void* vx,
                       const void* vy, const void* vz, const uint32_t* id) {
  static_cast<Base*>(h)->set_particles(n, c, off, vx, vy, vz, id);
}

void orc_set_ions(void* h, const double* ni, const double* gam) {
  Base* b = static_cast<Base*>(h);
  if (ni) std::copy(ni, ni + b->d.nn, b->ni.begin());
  if (gam) std::copy(gam, gam + b->d.nn, b->gam.begin());
}

// Grid state at the current step: cnt^n, n_i^n, Gamma, and the field of step n
// (phi, E, E' rounded to the particle precision) computed from them.
void orc_get_grid(void* h, int64_t* cnt, double* ni, double* gam, double* ne, double* phi,
                  double* E, void* Ep) {
  Base* b = static_cast<Base*>(h);
  const int nn = b->d.nn;
  std::vector<double> ne2(nn), rho2(nn), phi2(nn), E2(nn);
  const std::vector<double> nq = b->net_of(b->ni), gq = b->net_of(b->gam);
  field_solve(b->d, b->cnt.data(), nq.data(), b->V_cur, ne2.data(), rho2.data(),
              phi2.data(), E2.data());
  for (int j = 0; j < nn; ++j) {
    if (cnt) cnt[j] = b->cnt[j];
    if (ni) ni[j] = nq[j];
    if (gam) gam[j] = gq[j];
    if (ne) ne[j] = ne2[j];
    if (phi) phi[j] = phi2[j];
    if (E) E[j] = E2[j];
  }
  if (Ep) b->get_ep(Ep);
}

// counters: [coll[0..15], absorbed L, absorbed R, emitted L, emitted R,
//            created, overflow, see_clamped, n_acc, pushed]  (25 values)
void orc_get_counters(void* h, uint64_t* out) {
  Base* b = static_cast<Base*>(h);
  for (int k = 0; k < kMaxChannels; ++k) out[k] = b->ctr.coll[k];
  out[16] = b->ctr.absorbed[0];
  out[17] = b->ctr.absorbed[1];
  out[18] = b->ctr.emitted[0];
  out[19] = b->ctr.emitted[1];
  out[20] = b->ctr.created;
  out[21] = b->ctr.overflow;
  out[22] = b->ctr.see_clamped;
  out[23] = b->n_acc;
  out[24] = b->ctr.pushed;
}

// Density and flux of ion species s (ion model 4; s = 0 otherwise).
void orc_get_species(void* h, int s, double* ni, double* gam) {
  Base* b = static_cast<Base*>(h);
  const int nn = b->d.nn;
  for (int j = 0; j < nn; ++j) {
    if (ni) ni[j] = b->ni[(size_t)s * nn + j];
    if (gam) gam[j] = b->gam[(size_t)s * nn + j];
  }
}

// Mobility of species s at field E, and one drift-diffusion update of that
// species alone (in place) with a given E; returns its wall fluxes.
double orc_species_mobility(void* h, int s, double E) {
  Base* b = static_cast<Base*>(h);
  return species_mobility(b->d, b->d.sp[s], E);
}
void orc_fluid_species(void* h, int s, double* ni, double* gam, const double* E, double* gw) {
  Base* b = static_cast<Base*>(h);
  fluid_species(b->d, b->d.sp[s], ni, E, gam, gw);
}

void orc_get_accum(void* h, uint64_t* acc_cnt, double* acc_ni, uint64_t* eedf) {
  Base* b = static_cast<Base*>(h);
  if (acc_cnt) std::copy(b->acc_cnt.begin(), b->acc_cnt.end(), acc_cnt);
  if (acc_ni) std::copy(b->acc_ni.begin(), b->acc_ni.end(), acc_ni);
  if (eedf) std::copy(b->eedf.begin(), b->eedf.end(), eedf);
}

// Derived scalars: [dz, w, nu_max, Pmax, KE, invKE, kdz, delta, keedf, qm_dt,
//                   kappa, TN, M, nfloor]
void orc_get_derived(void* h, double* out) {
  const Derived& d = static_cast<Base*>(h)->d;
  const double v[] = {d.dz, d.w, d.nu_max, d.Pmax, d.KE, d.invKE, d.kdz,
                      d.delta, d.keedf, d.qm_dt, d.kappa, d.TN, d.M, d.nfloor};
  std::copy(v, v + 14, out);
}

// The cumulative collision-probability table (FP64, n_energy x K).
void orc_get_table(void* h, double* out) {
  const Derived& d = static_cast<Base*>(h)->d;
  std::copy(d.cum.begin(), d.cum.end(), out);
}

// ---- unit-level entry points used by the pins --------------------------

void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
}

// n uniforms of stream S(tag, id, step) in the given precision.
void orc_uniforms(uint64_t seed, uint32_t tag, uint32_t id, uint32_t step, int precision, int64_t n,
                  double* out) {
  Stream s(seed, tag, id, step);
  for (int64_t i = 0; i < n; ++i) out[i] = precision == 0 ? (double)uniform_f32(s) : uniform_f64(s);
}

void orc_thomas(int n, const double* a, const double* b, const double* c, const double* d,
                double* x) {
  thomas(n, a, b, c, d, x);
}

// The partitioned tridiagonal solve used by the field and the full fluid.
void orc_solve_tridiag(int n, const double* a, const double* b, const double* c, const double* d,
                       double* x) {
  solve_tridiag(n, a, b, c, d, x);
}

// [amplitude U of the coming levels, P_abs of the last period, completed
//  periods, steps per period, the current period's running sum]
void orc_get_power(void* h, double* out) {
  Base* b = static_cast<Base*>(h);
  out[0] = b->amp;
  out[1] = b->p_abs;
  out[2] = (double)b->rf_periods;
  out[3] = (double)b->rf_steps;
  out[4] = b->pw_sum;
}

void* orc_swarm_create(const orc_swarm_params* p) { return make_swarm(p); }
void orc_swarm_free(void* h) { delete static_cast<SwarmBase*>(h); }
void orc_swarm_run(void* h, int64_t n, int accumulate) {
  static_cast<SwarmBase*>(h)->run(n, accumulate);
}
void orc_swarm_get(void* h, int f, void* vx, void* vy, void* vz, double* avz, double* av2) {
  static_cast<SwarmBase*>(h)->get(f, vx, vy, vz, avz, av2);
}
// [sum of v_z, sum of |v|^2 over ions and accumulated steps, accumulated
//  steps, collisions, table overflows, step index]
void orc_swarm_sums(void* h, int f, double* out) {
  SwarmBase* b = static_cast<SwarmBase*>(h);
  out[0] = b->sum_vz(f);
  out[1] = b->sum_v2(f);
  out[2] = (double)b->n_acc[f];
  out[3] = (double)b->coll[f];
  out[4] = (double)b->over[f];
  out[5] = (double)b->step;
}
// normal deviates of stream (seed, tag, id, step): n pairs
void orc_normal_pairs(uint64_t seed, uint32_t tag, uint32_t id, uint32_t step, int n, int contract,
                      double* out) {
  Stream st(seed, tag, id, step);
  for (int k = 0; k < n; ++k) normal_pair(st, contract != 0, out[2 * k], out[2 * k + 1]);
}

int orc_field_partitions(int n) { return field_partitions(n); }
void orc_pcr_fma(int m, const double* a, const double* b, const double* c, const double* d,
                 double* x) {
  pcr_fma(m, a, b, c, d, x);
}

double orc_fit_ln(double x) { return fit_ln(x); }
double orc_fit_exp(double y) { return fit_exp(y); }
double orc_mobility_fit(double E, int contract) { return mobility_fit(E, contract != 0); }
double orc_nu_fit(double u, int contract) { return nu_fit(u, contract != 0); }

void orc_solve_tridiag_fma(int n, const double* a, const double* b, const double* c, const double* d,
                       double* x) {
  solve_tridiag_fma(n, a, b, c, d, x);
}

int orc_n_partitions(int n) { return n_partitions(n); }

// Field solve for a discharge's geometry with externally given cnt, n_i, V.
void orc_field(void* h, const int64_t* cnt, const double* ni, double V, double* phi, double* E) {
  Base* b = static_cast<Base*>(h);
  const int nn = b->d.nn;
  std::vector<double> ne2(nn), rho2(nn);
  field_solve(b->d, cnt, ni, V, ne2.data(), rho2.data(), phi, E);
}

// One ion-fluid update in place (n_i, Gamma) with a given E; returns wall fluxes.
void orc_fluid(void* h, double* ni, double* gam, const double* E, double* gw) {
  Base* b = static_cast<Base*>(h);
  if (b->p.ion_model == 0 || b->p.ion_model == 2)
    fluid_dd(b->d, b->p.mu_const, b->p.ion_model == 2, ni, E, gam, gw);
  else
    fluid_full(b->d, b->p.nu_const, b->p.ion_model == 3, ni, E, gam, gw);
}

// Push n particles (precision 0: float arrays, 1: double arrays) through
// `steps` leapfrog steps in a fixed E' (node array of length nc+1).  status[k]
// is 0 inside, 1/2 when removed through the left/right wall (then frozen).
void orc_push(int precision, int64_t n, int32_t* c, void* off, void* vz, const void* Ep, int nc,
              double kdz, int64_t steps, int32_t* status) {
  for (int64_t k = 0; k < n; ++k) status[k] = 0;
  for (int64_t s = 0; s < steps; ++s)
    for (int64_t k = 0; k < n; ++k) {
      if (status[k] != 0) continue;
      if (precision == 0)
        status[k] = push<float>(c[k], ((float*)off)[k], ((float*)vz)[k], (const float*)Ep, nc,
                                (float)kdz);
      else
        status[k] = push<double>(c[k], ((double*)off)[k], ((double*)vz)[k], (const double*)Ep, nc,
                                 kdz);
    }
}

// Collision step of a discharge's tables for n particles at step `step`
// (positions untouched).  channel[k] = -1 for no collision; child velocities
// written for ionizations (kid_v: n x 3, zero otherwise).
void orc_collide(void* h, int64_t n, const int32_t* c, const void* off, void* vx, void* vy,
                 void* vz, const uint32_t* id, uint32_t step, int32_t* channel, void* kid_v) {
  Base* b = static_cast<Base*>(h);
  if (b->p.precision == 0) {
    auto* D = static_cast<Discharge<float>*>(b);
    for (int64_t k = 0; k < n; ++k) {
      Particle<float> pt{c[k], ((const float*)off)[k], ((float*)vx)[k], ((float*)vy)[k],
                         ((float*)vz)[k], id[k]};
      Mcc<float> r = collide<float>(pt, D->q, b->p.seed, step);
      ((float*)vx)[k] = pt.vx;
      ((float*)vy)[k] = pt.vy;
      ((float*)vz)[k] = pt.vz;
      channel[k] = r.channel;
      float* kv = (float*)kid_v + 3 * k;
      kv[0] = r.child ? r.kid.vx : 0.f;
      kv[1] = r.child ? r.kid.vy : 0.f;
      kv[2] = r.child ? r.kid.vz : 0.f;
    }
  } else {
    auto* D = static_cast<Discharge<double>*>(b);
    for (int64_t k = 0; k < n; ++k) {
      Particle<double> pt{c[k], ((const double*)off)[k], ((double*)vx)[k], ((double*)vy)[k],
                          ((double*)vz)[k], id[k]};
      Mcc<double> r = collide<double>(pt, D->q, b->p.seed, step);
      ((double*)vx)[k] = pt.vx;
      ((double*)vy)[k] = pt.vy;
      ((double*)vz)[k] = pt.vz;
      channel[k] = r.channel;
      double* kv = (double*)kid_v + 3 * k;
      kv[0] = r.child ? r.kid.vx : 0.0;
      kv[1] = r.child ? r.kid.vy : 0.0;
      kv[2] = r.child ? r.kid.vz : 0.0;
    }
  }
}

// Unit sphere samples from stream S(tag 0, id, step), one per id.
void orc_sphere(int precision, uint64_t seed, int64_t n, const uint32_t* id, uint32_t step,
                double* out) {
  for (int64_t k = 0; k < n; ++k) {
    Stream s(seed, kTagElectron, id[k], step);
    if (precision == 0) {
      float v[3];
      sphere<float>(s, v);
      for (int i = 0; i < 3; ++i) out[3 * k + i] = v[i];
    } else {
      double v[3];
      sphere<double>(s, v);
      for (int i = 0; i < 3; ++i) out[3 * k + i] = v[i];
    }
  }
}

// CIC deposit of n particles into g (length nc+1).
void orc_deposit(int precision, int64_t n, const int32_t* c, const void* off, int64_t* g) {
  for (int64_t k = 0; k < n; ++k) {
    if (c[k] < 0) continue;
    if (precision == 0)
      deposit<float>(c[k], ((const float*)off)[k], g);
    else
      deposit<double>(c[k], ((const double*)off)[k], g);
  }
}

// Secondary emission of one side for wall flux F at step n: returns the number
// of emitted particles (<= cap) and writes their state.
int64_t orc_emit(void* h, int side, double F, uint32_t n, int32_t* c, void* off, void* vx, void* vy,
                 void* vz, int64_t cap) {
  Base* b = static_cast<Base*>(h);
  int64_t m = 0;
  if (b->p.precision == 0) {
    std::vector<Particle<float>> out;
    static_cast<Discharge<float>*>(b)->emit(side, F, n, out);
    for (auto& e : out) {
      if (m >= cap) break;
      c[m] = e.c;
      ((float*)off)[m] = e.off;
      ((float*)vx)[m] = e.vx;
      ((float*)vy)[m] = e.vy;
      ((float*)vz)[m] = e.vz;
      ++m;
    }
  } else {
    std::vector<Particle<double>> out;
    static_cast<Discharge<double>*>(b)->emit(side, F, n, out);
    for (auto& e : out) {
      if (m >= cap) break;
      c[m] = e.c;
      ((double*)off)[m] = e.off;
      ((double*)vx)[m] = e.vx;
      ((double*)vy)[m] = e.vy;
      ((double*)vz)[m] = e.vz;
      ++m;
    }
  }
  return m;
}

}  // extern "C"
