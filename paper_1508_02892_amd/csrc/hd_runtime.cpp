// Host runtime of the MI355X hybrid PIC/MCC stepper: parameter validation,
// derived constants and null-collision tables (FP64), the initial electron
// load, the device layout of each discharge, launch sequencing (with a
// captured hipGraph per sort interval) and the C ABI of include/hd.h.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hd.h"
#include "hd_internal.h"

namespace hd {

// kernel-side entry points (k_electron.hip, k_field.hip, k_sort.hip)
template <class P>
size_t electron_lds_bytes(int D, int tab_max, int nn_max, int nb1_max, int fluid_nn, int K_max,
                          int variant);
template <class P>
hipError_t launch_electron_impl(const Disch<P>* d_dev, int D, int grid, int tab_max, int nn_max,
                                int nb1_max, int fluid_nn, int K_max, int variant, hipStream_t s);
template <class P>
int electron_occupancy(int tab_max, int nn_max, int nb1_max, int fluid_nn, int K_max, int D,
                       int variant);
int electron_variants();
// The electron variant with nontemporal traffic of ids, cells and offsets
// (drain, then load; velocities left to the caches), and the size of
// MI355X's memory-side cache (MALL, the Infinity Cache): particle state
// beyond it streams from HBM on every step.
constexpr int kElecVariantStreaming = 5;
constexpr uint64_t kMallBytes = 256ull << 20;

// The wide form of electron variant v (kElecWide + v: the same kernel with
// 1,024-thread workgroups) where v's workgroups fit only one per CU (large
// grids) and the wide ones fit: sixteen waves per CU instead of eight.
template <class P>
int widen_variant(int v, int tab_max, int nn_max, int nb1_max, int fluid_nn, int K_max, int D) {
  if (v >= kElecWide) return v;
  if (electron_occupancy<P>(tab_max, nn_max, nb1_max, fluid_nn, K_max, D, v) != 1) return v;
  return electron_occupancy<P>(tab_max, nn_max, nb1_max, fluid_nn, K_max, D, v + kElecWide) >= 1
             ? v + kElecWide
             : v;
}
template <class P>
hipError_t finalize_set_lds(int nn_max);
template <class P>
hipError_t launch_sort_impl(const Disch<P>* d_dev, int D, int grid, int tile, int nc_max,
                            hipStream_t s);
template <class P>
hipError_t sort_set_lds(int nc_max, int D);
size_t sort_lds_bytes(int nc_max, int D);
template <class P>
hipError_t launch_checkpoint(const Disch<P>* d_dev, int D, int restore, int grid, hipStream_t s);
size_t sort_parts(size_t nc, size_t tiles);
template <class P>
hipError_t launch_set_steps(const Disch<P>* d_dev, int D, int64_t n, hipStream_t s);

namespace {

// CODATA 2018
constexpr double kE = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kKb = 1.380649e-23;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kPi = 3.14159265358979323846;

thread_local std::string g_err;

int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}

#define HD_TRY(expr)                                                                  \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess)                                                             \
      return fail(HD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));     \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Counter-based stream for the initial load (same Philox4x32-10 definition
// as on the device).
void philox_host(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, uint32_t k0, uint32_t k1,
                 uint32_t o[4]) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
  }
  o[0] = x0;
  o[1] = x1;
  o[2] = x2;
  o[3] = x3;
}

struct HostStream {
  uint32_t k0, k1, id, step, tag, blk = 0;
  uint32_t w[4];
  int pos = 4;
  HostStream(uint64_t seed, uint32_t tag_, uint32_t id_, uint32_t step_)
      : k0((uint32_t)seed), k1((uint32_t)(seed >> 32)), id(id_), step(step_), tag(tag_) {}
  uint32_t word() {
    if (pos == 4) {
      philox_host(id, step, blk, tag, k0, k1, w);
      blk += 1;
      pos = 0;
    }
    return w[pos++];
  }
  double u64() {
    const uint64_t hi = word();
    const uint64_t lo = word();
    return (double)(((hi << 32) | lo) >> 11) * 0x1p-53;
  }
};

// Steps per RF period, round(1 / (f dt)); 0 without a drive frequency.
int64_t rf_steps_of(const hd_params& p) {
  if (!(p.f_rf_Hz > 0)) return 0;
  const double r = 1.0 / (p.f_rf_Hz * p.dt_s);
  return r < 4.0e18 ? (int64_t)std::llround(r) : 0;
}

// Ion models that solve Eq (2.3) (tridiagonal scratch in LDS).
bool full_fluid(int32_t m) { return m == HD_ION_FULL_CONST_NU || m == HD_ION_FULL_FIT_NU; }

bool validate(const hd_params* p, std::string& why) {
  if (!p) return (why = "null params"), false;
  if (p->abi_version != HD_ABI_VERSION) return (why = "abi_version mismatch"), false;
  if (p->precision != HD_FP32 && p->precision != HD_FP64) return (why = "precision"), false;
  if (p->ion_model < HD_ION_DD_CONST_MU || p->ion_model > HD_ION_DD_SPECIES)
    return (why = "ion_model"), false;
  const bool multi = p->ion_model == HD_ION_DD_SPECIES;
  if (multi && (p->n_species < 1 || p->n_species > HD_MAX_SPECIES || !p->species))
    return (why = "HD_ION_DD_SPECIES needs 1 .. 4 species"), false;
  if (!multi && p->n_species != 0) return (why = "species are for HD_ION_DD_SPECIES"), false;
  if (multi)
    for (int q = 0; q < p->n_species; ++q) {
      const hd_ion_species& sp = p->species[q];
      if ((sp.charge != 1 && sp.charge != -1) || sp.n_mu < 2 || sp.n_mu > kMaxMu ||
          !sp.mu_m2_Vs || !(sp.m_amu > 0) || !(sp.en_lo_Td > 0) ||
          !(sp.en_hi_Td > sp.en_lo_Td) || !std::isfinite(sp.en_hi_Td) ||
          !(sp.init_fraction >= 0) || !std::isfinite(sp.init_fraction))
        return (why = "ion species " + std::to_string(q)), false;
      for (int i = 0; i < sp.n_mu; ++i)
        if (!(sp.mu_m2_Vs[i] >= 0) || !std::isfinite(sp.mu_m2_Vs[i]))
          return (why = "mobility table of species " + std::to_string(q)), false;
    }
  if (p->n_cells < 2 || p->n_cells > kMaxCells) return (why = "n_cells out of [2, 4096]"), false;
  if (p->n_energy < 2 || p->n_energy > (1 << 20)) return (why = "n_energy"), false;
  if (p->n_channels < 0 || p->n_channels > HD_MAX_CHANNELS) return (why = "n_channels"), false;
  if (p->n_channels > 0 && !p->channels) return (why = "channels missing"), false;
  for (int k = 0; k < p->n_channels; ++k) {
    const hd_xs_channel& c = p->channels[k];
    if (c.kind < HD_XS_ELASTIC || c.kind > HD_XS_ATTACHMENT || !c.sigma_m2 ||
        !(c.target_fraction >= 0) || !std::isfinite(c.target_fraction) ||
        !(c.target_mass_amu >= 0) || !std::isfinite(c.target_mass_amu))
      return (why = "channel " + std::to_string(k)), false;
    const int S = multi ? p->n_species : 1;
    if ((c.kind == HD_XS_IONIZATION || c.kind == HD_XS_ATTACHMENT) &&
        (c.product < 0 || c.product >= S))
      return (why = "channel " + std::to_string(k) + ": product species"), false;
    if (c.kind == HD_XS_IONIZATION && multi && p->species[c.product].charge != 1)
      return (why = "channel " + std::to_string(k) + ": ionization makes a positive ion"), false;
    if (c.kind == HD_XS_ATTACHMENT && (!multi || p->species[c.product].charge != -1))
      return (why = "channel " + std::to_string(k) + ": attachment makes a negative ion"), false;
    for (int i = 0; i < p->n_energy; ++i)
      if (!(c.sigma_m2[i] >= 0) || !std::isfinite(c.sigma_m2[i]))
        return (why = "cross section must be finite and non-negative"), false;
  }
  if (p->sort_every < 1 || p->eedf_every < 1 || p->n_eedf_bins < 1 || p->n_eedf_bins > 65536)
    return (why = "sort_every / eedf_every / n_eedf_bins"), false;
  if (p->n_macro < 0 || p->capacity < p->n_macro || p->capacity > (int64_t)2000000000)
    return (why = "n_macro / capacity"), false;
  if (!(p->gap_m > 0) || !(p->dt_s > 0) || !(p->inv_de_per_eV > 0) || !(p->eedf_emax_eV > 0))
    return (why = "gap / dt / energy grid"), false;
  if (!(p->load_lo >= 0) || !(p->load_hi <= 1) || !(p->load_hi > p->load_lo))
    return (why = "load interval"), false;
  if (p->n_macro > 0 && !(p->n_e0_m3 > 0)) return (why = "n_e0"), false;
  if (!(p->m_gas_amu > 0) || !(p->m_ion_amu > 0) || !(p->n_gas_m3 >= 0) || !(p->t_gas_K >= 0))
    return (why = "gas / ion parameters"), false;
  if (p->ion_model == HD_ION_FULL_CONST_NU && !(p->nu_const > 0)) return (why = "nu_const"), false;
  if (!(p->gamma_see >= 0) || !(p->e_sec_eV >= 0)) return (why = "emission parameters"), false;
  if (!(p->power_W_m2 >= 0) || !std::isfinite(p->power_W_m2) || !(p->power_alpha >= 0) ||
      !std::isfinite(p->power_alpha))
    return (why = "power control parameters"), false;
  if (p->power_W_m2 > 0 && rf_steps_of(*p) < 2)
    return (why = "power control needs an RF period of at least 2 steps"), false;
  return true;
}

size_t round_capacity(int64_t cap) {
  const size_t c = (size_t)std::max<int64_t>(cap, 1);
  return align_up(c, (size_t)kSortTile);  // also a multiple of kTile
}

// Byte layout of one discharge's device block.
struct Layout {
  size_t total = 0;
  size_t take(size_t bytes) {
    const size_t o = total;
    total = align_up(total + bytes, 256);
    return o;
  }
};

template <class P>
struct Offsets {
  size_t cell[2], off[2], vx[2], vy[2], vz[2], id[2];
  size_t kc, koff, kvx, kvy, kvz, chunk_kids, chunk_base, seg;
  size_t sc, soff, svx, svy, svz;
  size_t cnt[2], ion_src, ni, gam, mu, phi, E, Ep, scratch, acc_cnt, acc_ni, eedf;
  size_t ip, tab, hist, parts, tile_rng, st, volt, ckpt;
  size_t total;
};

template <class P>
Offsets<P> layout(const hd_params& p, int64_t volt_len) {
  Offsets<P> o;
  Layout L;
  const size_t C = round_capacity(p.capacity);
  const size_t nn = (size_t)p.n_cells + 1;
  for (int b = 0; b < 2; ++b) {
    o.cell[b] = L.take(C * 4);
    o.off[b] = L.take(C * sizeof(P));
    o.vx[b] = L.take(C * sizeof(P));
    o.vy[b] = L.take(C * sizeof(P));
    o.vz[b] = L.take(C * sizeof(P));
    o.id[b] = L.take(C * 4);
  }
  o.kc = L.take(C * 4);
  o.koff = L.take(C * sizeof(P));
  o.kvx = L.take(C * sizeof(P));
  o.kvy = L.take(C * sizeof(P));
  o.kvz = L.take(C * sizeof(P));
  o.chunk_kids = L.take(C / kSub * 4);
  o.chunk_base = L.take(C / kSub * 4);
  o.seg = L.take((size_t)kMaxSegs * 4);
  o.sc = L.take(2 * kSeeMax * 4);
  o.soff = L.take(2 * kSeeMax * sizeof(P));
  o.svx = L.take(2 * kSeeMax * sizeof(P));
  o.svy = L.take(2 * kSeeMax * sizeof(P));
  o.svz = L.take(2 * kSeeMax * sizeof(P));
  o.cnt[0] = L.take(nn * 8);
  o.cnt[1] = L.take(nn * 8);
  const size_t S = p.ion_model == HD_ION_DD_SPECIES ? (size_t)p.n_species : 1;
  o.ion_src = L.take(S * nn * 8);
  o.ni = L.take(S * nn * 8);
  o.gam = L.take(S * nn * 8);
  o.mu = L.take(S * kMaxMu * 8);
  o.phi = L.take(nn * 8);
  o.E = L.take(nn * 8);
  o.Ep = L.take(nn * sizeof(P));
  o.scratch = L.take(12 * nn * 8);
  o.acc_cnt = L.take(nn * 8);
  o.acc_ni = L.take(nn * 8);
  o.eedf = L.take(((size_t)p.n_eedf_bins + 1) * 8);
  o.ip = L.take(nn * 8);
  o.tab = L.take((size_t)p.n_energy * (size_t)std::max(p.n_channels, 1) * sizeof(P));
  o.hist = L.take((size_t)p.n_cells * (C / kSortTile) * 4);
  o.parts = L.take(sort_parts((size_t)p.n_cells, C / kSortTile) * 4);
  o.tile_rng = L.take(2 * (C / kSortTile) * 4);
  o.st = L.take(sizeof(State));
  o.ckpt = L.take((o.ip - o.cnt[0]) + sizeof(State));
  o.volt = L.take((size_t)volt_len * 8);
  o.total = L.total;
  return o;
}

constexpr int64_t kVoltInitial = 1 << 15;

// Everything the host keeps for one discharge.
template <class P>
struct Host {
  hd_params p{};
  std::vector<hd_xs_channel> ch;
  std::vector<std::vector<double>> sig;
  std::vector<hd_ion_species> sp;
  std::vector<std::vector<double>> mu;
  Disch<P> dd{};             // host copy of the device descriptor
  unsigned char* base = nullptr;
  size_t bytes = 0;
  int64_t volt_len = 0;
  int64_t volt_len0 = 0;     // entries of the drive table inside the block
  double* volt_dev = nullptr;
  int64_t host_step = 0;     // steps enqueued so far
  // derived FP64 values kept for moments
  double scale_in = 0, scale_wall = 0, keedf = 0;
};

template <class P>
void derive(Host<P>& h, std::vector<double>& ip, std::vector<P>& tab) {
  const hd_params& p = h.p;
  Disch<P>& d = h.dd;
  d.nc = p.n_cells;
  d.nn = p.n_cells + 1;
  d.ne = p.n_energy;
  d.K = p.n_channels;
  d.nbins = p.n_eedf_bins;
  d.sort_every = p.sort_every;
  d.eedf_every = p.eedf_every;
  d.ion_model = p.ion_model;
  d.seed = p.seed;
  const double dz = p.gap_m / p.n_cells;
  const double w =
      p.n_macro > 0 ? p.n_e0_m3 * (p.load_hi - p.load_lo) * p.gap_m / (double)p.n_macro : 0.0;
  d.dz = dz;
  d.L = p.gap_m;
  d.w = w;
  d.kp = dz * dz / kEps0;
  d.inv_dz = 1.0 / dz;
  d.inv_2dz = 0.5 / dz;
  d.hdz_eps = dz / (2.0 * kEps0);
  d.qm_dt = (-kE / kMe) * p.dt_s;
  d.scale_in = std::ldexp(w, -32) / dz;
  d.scale_wall = std::ldexp(w, -32) / (0.5 * dz);
  h.scale_in = d.scale_in;
  h.scale_wall = d.scale_wall;
  // Poisson pivots
  ip.assign(d.nn, 0.0);
  if (d.nc - 1 >= 1) {
    double den = 2.0;
    ip[1] = 1.0 / den;
    for (int j = 2; j <= d.nc - 1; ++j) {
      den = 2.0 - ip[j - 1];
      ip[j] = 1.0 / den;
    }
  }
  // ion fluid
  d.mu = p.mu_const;
  d.nu = p.nu_const;
  d.M = p.m_ion_amu * kAmu;
  const double mN = p.m_gas_amu * kAmu;
  d.TN = kKb * p.t_gas_K;
  d.kappa = (d.M + mN) / (5.0 * d.M + 3.0 * mN) * mN;
  d.mu_full = p.nu_const > 0 ? kE / (d.M * p.nu_const) : 0.0;
  d.dt = p.dt_s;
  d.dt_2dz = p.dt_s / (2.0 * dz);
  d.dt_dz = p.dt_s / dz;
  d.e_M_dt = kE * p.dt_s / d.M;
  d.dt_2dzM = p.dt_s / (2.0 * dz * d.M);
  d.hdt = 0.5 * p.dt_s;
  d.nfloor = 1e-10 * p.n_e0_m3;
  // drive: steps per RF period and the power control of Eq 2.9
  d.rf_steps = rf_steps_of(p);
  d.power_P0 = p.power_W_m2;
  d.power_alpha = p.power_alpha;
  // emission
  d.gamma_see = p.gamma_see;
  const double invKE = 2.0 * kE / kMe;
  d.see_v = std::sqrt(p.e_sec_eV * invKE);
  // null-collision tables: nu_k(E_i) = N_g sigma_k(E_i) sqrt(2 e E_i / m_e)
  const int ne = p.n_energy, K = p.n_channels;
  std::vector<double> nu((size_t)ne * K);
  double nu_max = 0.0;
  for (int i = 0; i < ne; ++i) {
    const double Ei = (double)i / p.inv_de_per_eV;
    const double v = std::sqrt(2.0 * kE * Ei / kMe);
    double tot = 0.0;
    for (int k = 0; k < K; ++k) {
      nu[(size_t)i * K + k] =
          (p.n_gas_m3 * p.channels[k].target_fraction) * p.channels[k].sigma_m2[i] * v;
      tot += nu[(size_t)i * K + k];
    }
    if (tot > nu_max) nu_max = tot;
  }
  const double Pmax = nu_max > 0 ? 1.0 - std::exp(-nu_max * p.dt_s) : 0.0;
  tab.assign((size_t)ne * std::max(K, 1), (P)0);
  for (int i = 0; i < ne; ++i) {
    double acc = 0.0;
    for (int k = 0; k < K; ++k) {
      acc += nu[(size_t)i * K + k];
      tab[(size_t)i * K + k] = (P)(nu_max > 0 ? Pmax * acc / nu_max : 0.0);
    }
  }
  d.Pmax = (P)Pmax;
  d.KE = (P)(0.5 * kMe / kE);
  d.invKE = (P)invKE;
  d.inv_dE = (P)p.inv_de_per_eV;
  d.kdz = (P)(p.dt_s / dz);
  d.delta = (P)(2.0 * kMe / (p.m_gas_amu * kAmu));
  for (int k = 0; k < K; ++k) {
    const double mt = p.channels[k].target_mass_amu > 0 ? p.channels[k].target_mass_amu
                                                         : p.m_gas_amu;
    d.delta_k[k] = (P)(2.0 * kMe / (mt * kAmu));
    d.product[k] = p.channels[k].product;
  }
  // ion species: one of charge +1 for the single-species models
  d.n_gas = p.n_gas_m3;
  const double mNs = p.m_gas_amu * kAmu;
  if (p.ion_model == HD_ION_DD_SPECIES) {
    d.S = p.n_species;
    for (int q = 0; q < d.S; ++q) {
      const hd_ion_species& sp = p.species[q];
      const double Ms = sp.m_amu * kAmu;
      d.Z[q] = sp.charge;
      d.n_mu[q] = sp.n_mu;
      d.kappa_s[q] = (Ms + mNs) / (5.0 * Ms + 3.0 * mNs) * mNs;
      d.mu_lo[q] = sp.en_lo_Td;
      d.mu_L0[q] = std::log(sp.en_lo_Td);
      d.mu_inv_dL[q] = (double)(sp.n_mu - 1) / (std::log(sp.en_hi_Td) - d.mu_L0[q]);
    }
  } else {
    d.S = 1;
    d.Z[0] = 1;
  }
  h.keedf = (double)p.n_eedf_bins / p.eedf_emax_eV;
  d.keedf = (P)h.keedf;
  d.ion_mask = 0;
  d.att_mask = 0;
  for (int k = 0; k < kMaxK; ++k) {
    d.thr[k] = k < K ? (P)p.channels[k].threshold_eV : (P)0;
    d.kind[k] = k < K ? p.channels[k].kind : 0;
    if (k < K && d.kind[k] == HD_XS_IONIZATION) d.ion_mask |= 1u << k;
    if (k < K && d.kind[k] == HD_XS_ATTACHMENT) d.att_mask |= 1u << k;
  }
}

// Initial load: stream (tag 1, id k, step 0); uniform position in
// [lo L, hi L), isotropic Maxwellian velocity (two polar-method pairs, the
// fourth deviate unused); then a stable sort by cell and the fixed-point
// deposit.
template <class P>
struct Loaded {
  std::vector<int32_t> cell;
  std::vector<P> off, vx, vy, vz;
  std::vector<uint32_t> id;
  std::vector<int64_t> cnt;
};

template <class P>
void load_one(const hd_params& p, double dz, double vth, int64_t k, int32_t& c, P& off, P& vx,
              P& vy, P& vz) {
  HostStream st(p.seed, 1u, (uint32_t)k, 0u);
  const double u0 = st.u64();
  const double z = p.gap_m * (p.load_lo + (p.load_hi - p.load_lo) * u0);
  const double s = z / dz;
  const double fl = std::floor(s);
  c = (int32_t)fl;
  off = (P)(s - fl);
  if (off == (P)1) {
    c = c + 1;
    off = (P)0;
  }
  double g[4];
  for (int pair = 0; pair < 2; ++pair) {
    double a, b, q;
    for (;;) {
      a = 2.0 * st.u64() - 1.0;
      b = 2.0 * st.u64() - 1.0;
      q = a * a + b * b;
      if (q < 1.0 && q > 0.0) break;
    }
    const double f = std::sqrt(-2.0 * std::log(q) / q);
    g[2 * pair] = a * f;
    g[2 * pair + 1] = b * f;
  }
  vx = (P)(vth * g[0]);
  vy = (P)(vth * g[1]);
  vz = (P)(vth * g[2]);
}

template <class P>
void load(const hd_params& p, double dz, Loaded<P>& out) {
  const int64_t N = p.n_macro;
  const int nc = p.n_cells;
  std::vector<int32_t> c0(N);
  std::vector<P> o0(N), x0(N), y0(N), z0(N);
  const double vth = std::sqrt(p.t_e0_eV * kE / kMe);
  unsigned nt = std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
  if (N < 65536) nt = 1;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    th.emplace_back([&, t]() {
      const int64_t a = N * t / nt, b = N * (t + 1) / nt;
      for (int64_t k = a; k < b; ++k) load_one<P>(p, dz, vth, k, c0[k], o0[k], x0[k], y0[k], z0[k]);
    });
  }
  for (auto& x : th) x.join();
  // stable counting sort by cell
  std::vector<int64_t> start(nc + 1, 0);
  for (int64_t k = 0; k < N; ++k) start[c0[k] + 1] += 1;
  for (int c = 0; c < nc; ++c) start[c + 1] += start[c];
  out.cell.resize(N);
  out.off.resize(N);
  out.vx.resize(N);
  out.vy.resize(N);
  out.vz.resize(N);
  out.id.resize(N);
  for (int64_t k = 0; k < N; ++k) {
    const int64_t o = start[c0[k]]++;
    out.cell[o] = c0[k];
    out.off[o] = o0[k];
    out.vx[o] = x0[k];
    out.vy[o] = y0[k];
    out.vz[o] = z0[k];
    out.id[o] = (uint32_t)k;
  }
  out.cnt.assign(nc + 1, 0);
  for (int64_t k = 0; k < N; ++k) {
    const int64_t W1 = (int64_t)std::rint(out.off[k] * (P)4294967296.0);
    out.cnt[out.cell[k]] += ((int64_t)1 << 32) - W1;
    out.cnt[out.cell[k] + 1] += W1;
  }
}

// Unit drive waveform at step n; the device scales it by the amplitude of
// the RF period (v_amp_V, or the power-controlled value of Eq 2.9).
double volt_at(const hd_params& p, int64_t n) {
  const double two_pi_f = 2.0 * kPi * p.f_rf_Hz;
  const double t = (double)n * p.dt_s;
  return std::sin(two_pi_f * t + p.phase_rad);
}

// Launch shapes chosen by the autotuner, per device and batch shape, for the
// life of the process (and, when HD_TUNE_CACHE names a file, across
// processes: one line "key variant electron_groups sort_groups append_groups
// sort_tile" per choice, the last line of a key winning; a line without the
// tile keeps the default tile).
std::mutex g_tune_mu;
std::map<std::string, hd_launch_config> g_tune;
bool g_tune_loaded = false;

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("HD_TUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream ss(line);
    std::string key;
    hd_launch_config c{};
    if (ss >> key >> c.electron_variant >> c.electron_groups >> c.sort_groups >> c.append_groups) {
      if (!(ss >> c.sort_tile)) c.sort_tile = 0;
      g_tune[key] = c;
    }
  }
}

bool tune_lookup(const std::string& key, hd_launch_config& out) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  out = it->second;
  return true;
}

void tune_store(const std::string& key, const hd_launch_config& c) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_load_locked();
  g_tune[key] = c;
  const char* path = std::getenv("HD_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  f << key << ' ' << c.electron_variant << ' ' << c.electron_groups << ' ' << c.sort_groups << ' '
    << c.append_groups << ' ' << c.sort_tile << '\n';
}

}  // namespace

// Device memory of a handle: carved from the caller's arena when the device
// context brings one (256-byte aligned, bump allocation, released with the
// handle), else from hipMalloc.
struct DevMem {
  unsigned char* arena = nullptr;
  size_t arena_bytes = 0, used = 0;
  std::vector<void*> owned;  // hipMalloc'd blocks
  int get(size_t n, void** p, const char* what) {
    if (arena) {
      const size_t o = align_up(used, 256);
      if (o > arena_bytes || n > arena_bytes - o) {
        *p = nullptr;
        return fail(HD_ENOMEM, std::string("arena too small for ") + what + " (" +
                                   std::to_string(o + n) + " bytes needed, " +
                                   std::to_string(arena_bytes) + " given)");
      }
      *p = arena + o;
      used = o + n;
      return HD_OK;
    }
    if (hipMalloc(p, n) != hipSuccess) {
      *p = nullptr;
      return fail(HD_ENOMEM, std::string("hipMalloc failed for ") + what + " (" +
                                 std::to_string(n) + " bytes)");
    }
    owned.push_back(*p);
    return HD_OK;
  }
  void release(void* p) {
    auto it = std::find(owned.begin(), owned.end(), p);
    if (it == owned.end()) return;  // arena memory: returned with the handle
    (void)hipFree(p);
    owned.erase(it);
  }
  ~DevMem() {
    for (void* p : owned) (void)hipFree(p);
  }
};

// ---------------------------------------------------------------------------
// Batch of discharges advanced together.
// ---------------------------------------------------------------------------
struct BatchBase {
  int precision = 0;
  int D = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int sort_every = 16;
  int grid_e = 0, grid_a = 0, grid_s = 0;
  int tile_s = kSortTile;   // items per sort tile (hd_launch_config)
  int tab_max = 0, nn_max = 0, nb1_max = 0, nc_max = 0, fluid_nn = 0, K_max = 1;
  int cus = 0;              // compute units of the device
  int elec_variant = 0;     // electron kernel variant (hd_launch_config)
  uint64_t state_bytes = 0; // initial particle state of all discharges
  hd_launch_config launch{};  // the applied shapes, defaults resolved
  std::string tune_key;     // the batch's key in the autotuner's cache
  int64_t host_step = 0;  // steps enqueued (all discharges advance together)
  int64_t graph_steps = 0;  // of those, steps replayed from captured graphs
  int64_t rollbacks = 0;    // capacity overflows rolled back
  bool replaying = false;   // re-running the steps of a rolled-back interval
  bool rolled_back = false; // stopped at an overflow; hd_grow clears it
  hipGraphExec_t graph = nullptr;       // one sort interval
  hipGraphExec_t graph_long = nullptr;  // kLongIntervals sort intervals
  // Intervals in the long graph: every graph launch leaves the GPU idle for
  // a few microseconds between the graphs, which the long one pays once per
  // kLongIntervals intervals.
  static constexpr int kLongIntervals = 8;
  void drop_graphs() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (graph_long) (void)hipGraphExecDestroy(graph_long);
    graph = nullptr;
    graph_long = nullptr;
  }
  bool graph_ok = true;   // capture supported
  int error = 0;
  hipStream_t own_stream = nullptr;  // created when the caller passes the null stream
  virtual ~BatchBase() {
    if (own_stream) (void)hipStreamDestroy(own_stream);
  }
};

template <class P>
struct Batch : BatchBase {
  std::vector<Host<P>> hs;
  Disch<P>* d_desc = nullptr;

  DevMem mem;

  ~Batch() override { drop_graphs(); }

  // Host-side preparation of one discharge (no device calls): derived
  // constants, tables, the initial load and the voltage table.
  struct Prepared {
    std::vector<double> ip, ni, vt, mu;
    std::vector<P> tab;
    Loaded<P> ld;
  };
  static void prepare_host(Host<P>& h, int64_t volt_len, Prepared& pr) {
    derive<P>(h, pr.ip, pr.tab);
    h.volt_len = volt_len;
    h.volt_len0 = volt_len;
    load<P>(h.p, h.dd.dz, pr.ld);
    const int nn = h.dd.nn, S = h.dd.S;
    pr.ni.assign((size_t)S * nn, 0.0);
    for (int j = 0; j < nn; ++j)
      pr.ni[j] = (double)pr.ld.cnt[j] * ((j == 0 || j == h.dd.nc) ? h.scale_wall : h.scale_in);
    // several species: species q starts at init_fraction_q of the electrons
    if (h.p.ion_model == HD_ION_DD_SPECIES)
      for (int q = S - 1; q >= 0; --q)
        for (int j = 0; j < nn; ++j)
          pr.ni[(size_t)q * nn + j] = h.p.species[q].init_fraction * pr.ni[j];
    pr.mu.assign((size_t)S * kMaxMu, 0.0);
    for (int q = 0; q < h.p.n_species; ++q)
      std::copy(h.mu[q].begin(), h.mu[q].end(), pr.mu.begin() + (size_t)q * kMaxMu);
    pr.vt.resize(volt_len);
    for (int64_t s = 0; s < volt_len; ++s) pr.vt[s] = volt_at(h.p, s);
  }

  // Allocates the discharge's device block and uploads the prepared state
  // (enqueued on the stream; the caller synchronises).
  static int upload_state(Host<P>& h, const Prepared& pr, hipStream_t stream, DevMem& mem) {
    const Offsets<P> o = layout<P>(h.p, h.volt_len);
    h.bytes = o.total;
    if (int rc = mem.get(h.bytes, (void**)&h.base, "a discharge's state")) {
      h.base = nullptr;
      return rc;
    }
    fill_pointers(h, o);
    HD_TRY(hipMemsetAsync(h.base, 0, h.bytes, stream));
    const Loaded<P>& ld = pr.ld;
    const size_t N = (size_t)h.p.n_macro;
    Disch<P>& d = h.dd;
    if (N) {
      HD_TRY(hipMemcpyAsync(d.cell[0], ld.cell.data(), N * 4, hipMemcpyHostToDevice, stream));
      HD_TRY(hipMemcpyAsync(d.off[0], ld.off.data(), N * sizeof(P), hipMemcpyHostToDevice, stream));
      HD_TRY(hipMemcpyAsync(d.vx[0], ld.vx.data(), N * sizeof(P), hipMemcpyHostToDevice, stream));
      HD_TRY(hipMemcpyAsync(d.vy[0], ld.vy.data(), N * sizeof(P), hipMemcpyHostToDevice, stream));
      HD_TRY(hipMemcpyAsync(d.vz[0], ld.vz.data(), N * sizeof(P), hipMemcpyHostToDevice, stream));
      HD_TRY(hipMemcpyAsync(d.id[0], ld.id.data(), N * 4, hipMemcpyHostToDevice, stream));
    }
    HD_TRY(hipMemcpyAsync(d.cnt[0], ld.cnt.data(), d.nn * 8, hipMemcpyHostToDevice, stream));
    HD_TRY(hipMemcpyAsync(d.ni, pr.ni.data(), pr.ni.size() * 8, hipMemcpyHostToDevice, stream));
    HD_TRY(hipMemcpyAsync((void*)d.mu_tab, pr.mu.data(), pr.mu.size() * 8, hipMemcpyHostToDevice,
                          stream));
    HD_TRY(hipMemcpyAsync((void*)d.ip, pr.ip.data(), d.nn * 8, hipMemcpyHostToDevice, stream));
    HD_TRY(hipMemcpyAsync((void*)d.tab, pr.tab.data(), pr.tab.size() * sizeof(P),
                          hipMemcpyHostToDevice, stream));
    HD_TRY(hipMemcpyAsync(h.volt_dev, pr.vt.data(), pr.vt.size() * 8, hipMemcpyHostToDevice,
                          stream));
    State st{};
    st.n_main = (uint32_t)N;
    st.next_id = (uint32_t)N;
    st.volt_amp = h.p.v_amp_V;
    // the first interval is checkpointed when it starts close to capacity
    // (the rule the sort applies to the later ones)
    st.ckpt_due = (uint64_t)N + 2ull * kSeeMax * (uint64_t)h.p.sort_every >
                  (uint64_t)h.p.capacity ? 1 : 0;
    st.prev_n_main = (uint32_t)N;
    HD_TRY(hipMemcpyAsync(d.st, &st, sizeof(State), hipMemcpyHostToDevice, stream));
    return HD_OK;
  }

  static void fill_pointers(Host<P>& h, const Offsets<P>& o) {
    unsigned char* b = h.base;
    Disch<P>& d = h.dd;
    const size_t C = round_capacity(h.p.capacity);
    d.capacity = (uint32_t)h.p.capacity;  // limit; buffers are rounded up to C
    d.cap_sub = (uint32_t)(C / kSub);
    d.sort_tiles_max = (uint32_t)(C / kSortTile);
    for (int i = 0; i < 2; ++i) {
      d.cell[i] = (int32_t*)(b + o.cell[i]);
      d.off[i] = (P*)(b + o.off[i]);
      d.vx[i] = (P*)(b + o.vx[i]);
      d.vy[i] = (P*)(b + o.vy[i]);
      d.vz[i] = (P*)(b + o.vz[i]);
      d.id[i] = (uint32_t*)(b + o.id[i]);
      d.cnt[i] = (int64_t*)(b + o.cnt[i]);
    }
    d.kc = (int32_t*)(b + o.kc);
    d.koff = (P*)(b + o.koff);
    d.kvx = (P*)(b + o.kvx);
    d.kvy = (P*)(b + o.kvy);
    d.kvz = (P*)(b + o.kvz);
    d.chunk_kids = (uint32_t*)(b + o.chunk_kids);
    d.chunk_base = (uint32_t*)(b + o.chunk_base);
    d.seg = (uint32_t*)(b + o.seg);
    d.sc = (int32_t*)(b + o.sc);
    d.soff = (P*)(b + o.soff);
    d.svx = (P*)(b + o.svx);
    d.svy = (P*)(b + o.svy);
    d.svz = (P*)(b + o.svz);
    d.ion_src = (int64_t*)(b + o.ion_src);
    d.ni = (double*)(b + o.ni);
    d.gam = (double*)(b + o.gam);
    d.mu_tab = (const double*)(b + o.mu);
    d.phi = (double*)(b + o.phi);
    d.E = (double*)(b + o.E);
    d.Ep = (P*)(b + o.Ep);
    d.scratch = (double*)(b + o.scratch);
    d.acc_cnt = (uint64_t*)(b + o.acc_cnt);
    d.acc_ni = (double*)(b + o.acc_ni);
    d.eedf = (uint64_t*)(b + o.eedf);
    d.ip = (const double*)(b + o.ip);
    d.tab = (const P*)(b + o.tab);
    d.hist = (uint32_t*)(b + o.hist);
    d.bin_start = (uint32_t*)(b + o.parts);
    d.tile_rng = (int32_t*)(b + o.tile_rng);
    d.st = (State*)(b + o.st);
    d.ckpt = b + o.ckpt;
    d.grid_bytes = o.ip - o.cnt[0];
    h.volt_dev = (double*)(b + o.volt);
    d.volt = h.volt_dev;
    d.volt_len = h.volt_len;
  }

  int create(const hd_params* const* params, int n, const hd_device_ctx* ctx) {
    D = n;
    stream = ctx ? (hipStream_t)ctx->stream : nullptr;
    device = ctx ? ctx->device : 0;
    if (ctx && ctx->arena) {
      if ((uintptr_t)ctx->arena % 256 != 0) return fail(HD_EINVAL, "arena must be 256-byte aligned");
      mem.arena = (unsigned char*)ctx->arena;
      mem.arena_bytes = ctx->arena_bytes;
    }
    HD_TRY(hipSetDevice(device));
    if (!stream) {  // the legacy default stream cannot be captured into a graph
      HD_TRY(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
      stream = own_stream;
    }
    hs.resize(n);
    for (int i = 0; i < n; ++i) {
      Host<P>& h = hs[i];
      h.p = *params[i];
      h.sig.resize(h.p.n_channels);
      h.ch.resize(h.p.n_channels);
      for (int k = 0; k < h.p.n_channels; ++k) {
        h.sig[k].assign(h.p.channels[k].sigma_m2, h.p.channels[k].sigma_m2 + h.p.n_energy);
        h.ch[k] = h.p.channels[k];
        h.ch[k].sigma_m2 = h.sig[k].data();
      }
      h.p.channels = h.ch.empty() ? nullptr : h.ch.data();
      h.sp.resize(h.p.n_species);
      h.mu.resize(h.p.n_species);
      for (int q = 0; q < h.p.n_species; ++q) {
        h.mu[q].assign(h.p.species[q].mu_m2_Vs, h.p.species[q].mu_m2_Vs + h.p.species[q].n_mu);
        h.sp[q] = h.p.species[q];
        h.sp[q].mu_m2_Vs = h.mu[q].data();
      }
      h.p.species = h.sp.empty() ? nullptr : h.sp.data();
      tab_max = std::max(tab_max, h.p.n_energy * std::max(1, h.p.n_channels));
      K_max = std::max(K_max, h.p.n_channels);
      nn_max = std::max(nn_max, h.p.n_cells + 1);
      nc_max = std::max(nc_max, h.p.n_cells);
      nb1_max = std::max(nb1_max, h.p.n_eedf_bins + 1);
      if (full_fluid(h.p.ion_model)) fluid_nn = std::max(fluid_nn, h.p.n_cells + 1);
    }
    sort_every = hs[0].p.sort_every;
    // launch geometry
    hipDeviceProp_t prop;
    HD_TRY(hipGetDeviceProperties(&prop, device));
    const size_t lds = electron_lds_bytes<P>(D, tab_max, nn_max, nb1_max, fluid_nn, K_max, 0);
    if (lds > (size_t)prop.sharedMemPerBlock)
      return fail(HD_EINVAL, "electron kernel needs " + std::to_string(lds) +
                                 " B of LDS, device allows " +
                                 std::to_string(prop.sharedMemPerBlock));
    if (sort_lds_bytes(nc_max, D) > (size_t)prop.sharedMemPerBlock)
      return fail(HD_EINVAL, "sort LDS too large");
    HD_TRY(sort_set_lds<P>(nc_max, D));
    HD_TRY(finalize_set_lds<P>(nn_max));
    cus = prop.multiProcessorCount;
    {
      int64_t slots = 0;
      for (const auto& h : hs) slots += h.p.capacity;
      int lg = 0;
      while (((int64_t)1 << lg) < slots) ++lg;
      int models = 0;
      for (const auto& h : hs) models |= 1 << h.p.ion_model;
      std::ostringstream k;
      k << prop.gcnArchName << ":" << cus << "/p" << precision << "/D" << D << "/n2^" << lg
        << "/nc" << nc_max << "/K" << K_max << "/m" << models;
      tune_key = k.str();
    }
    // Untuned default: nontemporal traffic of ids, cells and offsets once the
    // initial particle state is larger than the MALL, which it then cannot
    // stay in.
    hd_launch_config lc0{};
    {
      uint64_t bytes = 0;
      for (const auto& h : hs) bytes += (uint64_t)h.p.n_macro * (8u + 4u * sizeof(P));
      state_bytes = bytes;
      if (bytes > kMallBytes) lc0.electron_variant = kElecVariantStreaming;
      lc0.electron_variant = widen_variant<P>(lc0.electron_variant, tab_max, nn_max, nb1_max,
                                              fluid_nn, K_max, D);
    }
    hd_launch_config lc{};
    if (!tune_lookup(tune_key, lc) || apply_launch(lc) != HD_OK) {
      lc = lc0;
      const int rc = apply_launch(lc);
      if (rc) return rc;
    }
    // per-discharge state
    for (int i = 0; i < n; ++i) {
      Prepared pr;
      prepare_host(hs[i], kVoltInitial, pr);
      const int rc = upload_state(hs[i], pr, stream, mem);
      if (rc) return rc;
      HD_TRY(hipStreamSynchronize(stream));
    }
    if (int rc = mem.get(sizeof(Disch<P>) * D, (void**)&d_desc, "the discharge descriptors"))
      return rc;
    HD_TRY(upload_desc());
    HD_TRY(launch_finalize<P>(d_desc, D, 1, nn_max, 0, stream));
    HD_TRY(hipStreamSynchronize(stream));
    for (int i = 0; i < D; ++i) {  // the field of step 0 must be finite
      State st;
      HD_TRY(hipMemcpy(&st, hs[i].dd.st, sizeof(State), hipMemcpyDeviceToHost));
      if (st.error) return fail(st.error, "discharge " + std::to_string(i) + ": " + error_text(st));
    }
    return HD_OK;
  }

  hipError_t upload_desc() {
    std::vector<Disch<P>> v(D);
    for (int i = 0; i < D; ++i) v[i] = hs[i].dd;
    hipError_t e = hipMemcpyAsync(d_desc, v.data(), sizeof(Disch<P>) * D, hipMemcpyHostToDevice,
                                  stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(stream);
  }

  // Make every discharge's voltage table cover steps [0, upto].
  int ensure_volt(int64_t upto) {
    bool changed = false;
    for (auto& h : hs) {
      if (upto < h.volt_len) continue;
      int64_t len = h.volt_len;
      while (len <= upto) len *= 2;
      double* nv = nullptr;
      // earlier tables stay allocated: launches already enqueued may read them
      if (int rc = mem.get((size_t)len * 8, (void**)&nv, "the drive table")) return rc;
      std::vector<double> vt(len);
      for (int64_t s = 0; s < len; ++s) vt[s] = volt_at(h.p, s);
      HD_TRY(hipMemcpy(nv, vt.data(), (size_t)len * 8, hipMemcpyHostToDevice));
      h.volt_dev = nv;
      h.volt_len = len;
      h.dd.volt = nv;
      h.dd.volt_len = len;
      changed = true;
    }
    if (changed) {
      HD_TRY(hipStreamSynchronize(stream));
      HD_TRY(upload_desc());
      drop_graphs();
    }
    return HD_OK;
  }

  // Resolves and applies a launch configuration (0 fields: defaults).
  int apply_launch(const hd_launch_config& in) {
    hd_launch_config c = in;
    if (c.electron_variant < 0 || c.electron_variant >= electron_variants())
      return fail(HD_EINVAL, "electron_variant out of range");
    const int occ =
        electron_occupancy<P>(tab_max, nn_max, nb1_max, fluid_nn, K_max, D, c.electron_variant);
    if (occ < 1) return fail(HD_EINVAL, "this electron kernel variant cannot be resident");
    if (c.electron_groups == 0) c.electron_groups = std::min(cus * occ, (int)kMaxSegs);
    if (c.sort_groups == 0) c.sort_groups = cus * 4;
    if (c.append_groups == 0) c.append_groups = std::max(1, cus / 4);
    if (c.sort_tile == 0) c.sort_tile = kSortTile;
    if (c.sort_tile != kSortTile && c.sort_tile != 2 * kSortTile)
      return fail(HD_EINVAL, "sort_tile must be 4096 or 8192");
    if (c.electron_groups < 1 || c.electron_groups > kMaxSegs)
      return fail(HD_EINVAL, "electron_groups out of range");
    if (c.sort_groups < 1 || c.sort_groups > 65536)
      return fail(HD_EINVAL, "sort_groups out of range");
    if (c.append_groups < 1 || c.append_groups > cus)
      return fail(HD_EINVAL, "append_groups out of range");
    elec_variant = c.electron_variant;
    grid_e = D + c.electron_groups;
    grid_s = c.sort_groups;
    tile_s = c.sort_tile;
    grid_a = c.append_groups;
    launch = c;
    drop_graphs();  // captured with the old shapes
    return HD_OK;
  }

  // One step; at an interval's start (ckpt) the checkpoint launch first.
  hipError_t enqueue_step(bool with_sort, bool ckpt) {
    hipError_t e = hipSuccess;
    if (ckpt) e = launch_checkpoint<P>(d_desc, D, 0, std::max(1, cus * 2), stream);
    if (e != hipSuccess) return e;
    e = launch_electron_impl<P>(d_desc, D, grid_e, tab_max, nn_max, nb1_max, fluid_nn, K_max,
                                elec_variant, stream);
    if (e != hipSuccess) return e;
    e = launch_finalize<P>(d_desc, D, 0, nn_max, grid_a, stream);
    if (e != hipSuccess) return e;
    if (with_sort) e = launch_sort_impl<P>(d_desc, D, grid_s, tile_s, nc_max, stream);
    return e;
  }

  // Captures `intervals` sort intervals of steps into out; on failure the
  // handle falls back to direct launches of the same kernels.
  int capture(hipGraphExec_t& out, int intervals) {
    hipGraph_t g = nullptr;
    HD_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int s = 0; s < intervals * sort_every && e == hipSuccess; ++s)
      e = enqueue_step(s % sort_every == sort_every - 1, s % sort_every == 0);
    hipError_t e2 = hipStreamEndCapture(stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      graph_ok = false;
      return HD_OK;
    }
    e = hipGraphInstantiate(&out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      out = nullptr;
      graph_ok = false;
    }
    return HD_OK;
  }

  int step(int64_t n) {
    if (n < 0) return fail(HD_EINVAL, "n_steps < 0");
    if (error) return fail(error, "handle is in an error state");
    if (rolled_back)
      return fail(HD_ECAPACITY, "stopped at a capacity overflow: hd_grow first");
    if (n == 0) return HD_OK;
    const int64_t target = host_step + n;
    int rc = ensure_volt(target + 1);
    if (rc) return rc;
    HD_TRY(launch_set_steps<P>(d_desc, D, n, stream));
    while (host_step < target) {
      const int64_t left = target - host_step;
      if (host_step % sort_every == 0 && left >= sort_every && graph_ok && use_graph) {
        if (!graph) {  // both graphs at once, so that neither is captured mid-run
          rc = capture(graph, 1);
          if (rc == HD_OK && graph_ok) rc = capture(graph_long, kLongIntervals);
          if (rc) return rc;
          if (!graph || !graph_long) {
            drop_graphs();
            continue;
          }
        }
        const bool lng = left >= (int64_t)kLongIntervals * sort_every;
        HD_TRY(hipGraphLaunch(lng ? graph_long : graph, stream));
        const int64_t k = (int64_t)(lng ? kLongIntervals : 1) * sort_every;
        host_step += k;
        graph_steps += k;
      } else {
        const bool srt = ((host_step + 1) % sort_every) == 0;
        HD_TRY(enqueue_step(srt, host_step % sort_every == 0 && !replaying));
        host_step += 1;
      }
    }
    return HD_OK;
  }
  bool use_graph = true;

  static std::string error_text(const State& st) {
    const std::string at = " in step " + std::to_string(st.error_step);
    switch (st.error) {
      case HD_ECAPACITY:
        return "particle capacity exceeded" + at + " (no checkpoint of the interval: the handle stops)";
      case HD_ENUMERIC:
        return "the field after step " + std::to_string(st.error_step) + " is not finite";
      case HD_ESYNC:
        return "the append workgroups timed out waiting for the end-of-step workgroup";
      default:
        return "device reported error " + std::to_string(st.error);
    }
  }

  int sync_state(int i, State& st) {
    HD_TRY(hipStreamSynchronize(stream));
    HD_TRY(hipMemcpy(&st, hs[i].dd.st, sizeof(State), hipMemcpyDeviceToHost));
    if (st.error == HD_ECAPACITY && D == 1 && st.ckpt_valid && st.ckpt_step <= st.error_step)
      return rollback(st);
    if (st.error) {
      error = st.error;
      return fail(st.error, error_text(st));
    }
    return HD_OK;
  }

  // A capacity overflow of a single discharge with a checkpoint of its
  // interval: restore the checkpoint and replay the steps before the
  // overflowing one (the same launches, so the same run bit for bit); the
  // handle then stands at the last complete step.
  int rollback(State& st) {
    const int64_t target = st.error_step;
    HD_TRY(launch_checkpoint<P>(d_desc, D, 1, std::max(1, cus * 2), stream));
    HD_TRY(hipStreamSynchronize(stream));
    HD_TRY(hipMemcpy(&st, hs[0].dd.st, sizeof(State), hipMemcpyDeviceToHost));
    host_step = st.step;
    const int64_t n = target - host_step;
    if (n > 0) {
      HD_TRY(launch_set_steps<P>(d_desc, D, n, stream));
      replaying = true;
      hipError_t e = hipSuccess;
      for (int64_t k = 0; k < n && e == hipSuccess; ++k) {
        e = enqueue_step(((host_step + 1) % sort_every) == 0, false);
        host_step += 1;
      }
      replaying = false;
      HD_TRY(e);
      HD_TRY(hipStreamSynchronize(stream));
      HD_TRY(hipMemcpy(&st, hs[0].dd.st, sizeof(State), hipMemcpyDeviceToHost));
    }
    if (st.error || st.step != target) {
      error = st.error ? st.error : HD_EDEVICE;
      return fail(error, "rolling back the capacity overflow failed");
    }
    rollbacks += 1;
    rolled_back = true;
    return fail(HD_ECAPACITY, "particle capacity exceeded in step " + std::to_string(target) +
                                  "; rolled back to the end of step " + std::to_string(target - 1) +
                                  " (hd_grow, then hd_step)");
  }

  // ---- snapshot and resume of a single discharge --------------------------
  // The run's whole state at a step boundary: the state record, the particle
  // slots in use and the grids (deposits, ion densities and fluxes, fields,
  // run sums, EEDF).  The random streams are keyed by particle id and step,
  // so nothing else is needed for a resumed run to continue bit for bit as
  // the uninterrupted one.  A snapshot is restored only into a handle of the
  // same parameters (capacity aside), checked by a fingerprint of them.
  struct SaveHead {
    char magic[8];
    uint64_t fingerprint;
    int32_t abi, p_bytes;
    uint64_t state_bytes, n_main, grid_bytes, total;
  };
  static constexpr char kSaveMagic[8] = {'H', 'D', 'S', 'A', 'V', 'E', '0', '1'};

  uint64_t fingerprint() const {  // FNV-1a over the parameters and their tables
    const Host<P>& h = hs[0];
    uint64_t fp = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t n) {
      const unsigned char* c = static_cast<const unsigned char*>(p);
      for (size_t i = 0; i < n; ++i) fp = (fp ^ c[i]) * 1099511628211ull;
    };
    hd_params q = h.p;  // no padding: 10 int32, 3 64-bit integers, doubles, pointers
    q.capacity = 0;
    q.channels = nullptr;
    q.species = nullptr;
    mix(&q, sizeof q);
    for (size_t k = 0; k < h.ch.size(); ++k) {
      hd_xs_channel c = h.ch[k];
      c.sigma_m2 = nullptr;
      mix(&c, sizeof c);
      mix(h.sig[k].data(), h.sig[k].size() * sizeof(double));
    }
    for (size_t k = 0; k < h.sp.size(); ++k) {
      hd_ion_species c = h.sp[k];
      c.mu_m2_Vs = nullptr;
      mix(&c, sizeof c);
      mix(h.mu[k].data(), h.mu[k].size() * sizeof(double));
    }
    return fp;
  }

  int save(void* out, size_t cap, size_t* used) {
    if (D != 1) return fail(HD_EINVAL, "hd_save is for single discharges");
    if (!used) return fail(HD_EINVAL, "null size output");
    if (error) return fail(error, "handle is in an error state");
    State st;
    if (int rc = sync_state(0, st)) return rc;
    if (rolled_back) return fail(HD_ECAPACITY, "stopped at a capacity overflow: hd_grow first");
    const Host<P>& h = hs[0];
    const Offsets<P> o = layout<P>(h.p, h.volt_len0);
    SaveHead hd{};
    std::memcpy(hd.magic, kSaveMagic, 8);
    hd.fingerprint = fingerprint();
    hd.abi = HD_ABI_VERSION;
    hd.p_bytes = (int32_t)sizeof(P);
    hd.state_bytes = sizeof(State);
    hd.n_main = st.n_main;
    hd.grid_bytes = o.ip - o.cnt[0];
    hd.total = sizeof(SaveHead) + hd.state_bytes + hd.n_main * (8 + 4 * sizeof(P)) + hd.grid_bytes;
    *used = hd.total;
    if (!out) return HD_OK;  // size query
    if (cap < hd.total) return fail(HD_EINVAL, "snapshot buffer smaller than " + std::to_string(hd.total) + " bytes");
    unsigned char* w = static_cast<unsigned char*>(out);
    std::memcpy(w, &hd, sizeof hd);
    w += sizeof hd;
    std::memcpy(w, &st, sizeof st);
    w += sizeof st;
    const int b = st.buf;
    const size_t n = hd.n_main;
    auto get = [&](size_t off, size_t bytes) {
      hipError_t e = hipMemcpy(w, h.base + off, bytes, hipMemcpyDeviceToHost);
      w += bytes;
      return e;
    };
    HD_TRY(get(o.cell[b], n * 4));
    HD_TRY(get(o.off[b], n * sizeof(P)));
    HD_TRY(get(o.vx[b], n * sizeof(P)));
    HD_TRY(get(o.vy[b], n * sizeof(P)));
    HD_TRY(get(o.vz[b], n * sizeof(P)));
    HD_TRY(get(o.id[b], n * 4));
    HD_TRY(get(o.cnt[0], hd.grid_bytes));
    return HD_OK;
  }

  int restore(const void* in, size_t bytes) {
    if (D != 1) return fail(HD_EINVAL, "hd_restore is for single discharges");
    if (!in || bytes < sizeof(SaveHead)) return fail(HD_EINVAL, "not a snapshot");
    if (error) return fail(error, "handle is in an error state");
    SaveHead hd;
    std::memcpy(&hd, in, sizeof hd);
    if (std::memcmp(hd.magic, kSaveMagic, 8) != 0 || hd.abi != HD_ABI_VERSION ||
        hd.p_bytes != (int32_t)sizeof(P) || hd.state_bytes != sizeof(State))
      return fail(HD_EINVAL, "not a snapshot of this library and precision");
    if (hd.fingerprint != fingerprint())
      return fail(HD_EINVAL, "snapshot of a discharge with other parameters");
    Host<P>& h = hs[0];
    const Offsets<P> o = layout<P>(h.p, h.volt_len0);
    if (hd.grid_bytes != o.ip - o.cnt[0] ||
        hd.total != sizeof(SaveHead) + hd.state_bytes + hd.n_main * (8 + 4 * sizeof(P)) + hd.grid_bytes)
      return fail(HD_EINVAL, "inconsistent snapshot");
    if (bytes < hd.total) return fail(HD_EINVAL, "truncated snapshot");
    const unsigned char* r = static_cast<const unsigned char*>(in) + sizeof hd;
    State st;
    std::memcpy(&st, r, sizeof st);
    r += sizeof st;
    const size_t n = hd.n_main, cap_slots = round_capacity(h.p.capacity);
    if (n != st.n_main || st.error || (st.buf != 0 && st.buf != 1) || (st.cbuf != 0 && st.cbuf != 1))
      return fail(HD_EINVAL, "inconsistent snapshot");
    if (n > cap_slots) return fail(HD_ECAPACITY, "snapshot needs " + std::to_string(n) + " particle slots (hd_grow first)");
    HD_TRY(hipStreamSynchronize(stream));
    const int b = st.buf;
    auto put = [&](size_t off, size_t bytes) {
      hipError_t e = hipMemcpy(h.base + off, r, bytes, hipMemcpyHostToDevice);
      r += bytes;
      return e;
    };
    HD_TRY(put(o.cell[b], n * 4));
    HD_TRY(put(o.off[b], n * sizeof(P)));
    HD_TRY(put(o.vx[b], n * sizeof(P)));
    HD_TRY(put(o.vy[b], n * sizeof(P)));
    HD_TRY(put(o.vz[b], n * sizeof(P)));
    HD_TRY(put(o.id[b], n * 4));
    HD_TRY(put(o.cnt[0], hd.grid_bytes));
    st.steps_left = 0;
    st.ckpt_valid = 0;
    st.ckpt_due = (uint64_t)n + 2ull * kSeeMax * (uint64_t)sort_every > (uint64_t)cap_slots ? 1 : 0;
    HD_TRY(hipMemcpy(h.dd.st, &st, sizeof(State), hipMemcpyHostToDevice));
    host_step = st.step;
    rolled_back = false;
    drop_graphs();  // a graph holds no step-dependent input, but start clean
    return ensure_volt(host_step + 1);
  }

  // Raises the capacity of a single discharge: a new block of the larger
  // layout, the live state copied over, the old block released.
  int grow(int64_t cap) {
    if (D != 1) return fail(HD_EINVAL, "hd_grow is for single discharges");
    if (error) return fail(error, "handle is in an error state");
    Host<P>& h = hs[0];
    if (cap < h.p.capacity) return fail(HD_EINVAL, "new capacity below the current one");
    hd_params p2 = h.p;
    p2.capacity = cap;
    std::string why;
    if (!validate(&p2, why)) return fail(HD_EINVAL, why);
    HD_TRY(hipStreamSynchronize(stream));
    State st;
    HD_TRY(hipMemcpy(&st, h.dd.st, sizeof(State), hipMemcpyDeviceToHost));
    const Offsets<P> oo = layout<P>(h.p, h.volt_len0), on = layout<P>(p2, h.volt_len0);
    unsigned char* nb = nullptr;
    if (int rc = mem.get(on.total, (void**)&nb, "the grown state")) return rc;
    unsigned char* ob = h.base;
    HD_TRY(hipMemsetAsync(nb, 0, on.total, stream));
    const size_t n = st.n_main, b = (size_t)st.buf;
    auto cp = [&](size_t dst, size_t src, size_t bytes) {
      return hipMemcpyAsync(nb + dst, ob + src, bytes, hipMemcpyDeviceToDevice, stream);
    };
    HD_TRY(cp(on.cell[b], oo.cell[b], n * 4));
    HD_TRY(cp(on.off[b], oo.off[b], n * sizeof(P)));
    HD_TRY(cp(on.vx[b], oo.vx[b], n * sizeof(P)));
    HD_TRY(cp(on.vy[b], oo.vy[b], n * sizeof(P)));
    HD_TRY(cp(on.vz[b], oo.vz[b], n * sizeof(P)));
    HD_TRY(cp(on.id[b], oo.id[b], n * 4));
    // grids, run sums and tables keep their internal layout
    HD_TRY(cp(on.cnt[0], oo.cnt[0], oo.hist - oo.cnt[0]));
    HD_TRY(cp(on.volt, oo.volt, (size_t)h.volt_len0 * 8));
    st.ckpt_valid = 0;
    st.ckpt_due = (uint64_t)n + 2ull * kSeeMax * (uint64_t)sort_every > (uint64_t)cap ? 1 : 0;
    HD_TRY(hipMemcpyAsync(nb + on.st, &st, sizeof(State), hipMemcpyHostToDevice, stream));
    HD_TRY(hipStreamSynchronize(stream));
    double* ext = h.volt_dev != (double*)(ob + oo.volt) ? h.volt_dev : nullptr;
    h.p.capacity = cap;
    h.base = nb;
    h.bytes = on.total;
    fill_pointers(h, on);
    if (ext) {  // an extended drive table stays where it is
      h.volt_dev = ext;
      h.dd.volt = ext;
    }
    HD_TRY(upload_desc());
    mem.release(ob);
    drop_graphs();
    rolled_back = false;
    return HD_OK;
  }

  int moments(int i, hd_moment_set* m) {
    if (i < 0 || i >= D || !m) return fail(HD_EINVAL, "bad index or output");
    State st;
    const int rc = sync_state(i, st);
    const int rc2 = fill_moments(hs[i], st, m);
    m->graph_steps = graph_steps;
    m->rollbacks = rollbacks;
    return rc ? rc : rc2;
  }

  // Moments of a discharge whose stream is idle, given its State.
  static int fill_moments(const Host<P>& h, const State& st, hd_moment_set* m) {
    const Disch<P>& d = h.dd;
    const int rc = HD_OK;
    const int nn = d.nn;
    m->step = st.step;
    m->n_slots = st.n_main;
    m->n_nodes = nn;
    m->n_channels = d.K;
    m->n_eedf_bins = d.nbins;
    m->error = st.error;
    for (int k = 0; k < HD_MAX_CHANNELS; ++k) m->coll[k] = k < kMaxK ? st.coll[k] : 0;
    m->absorbed[0] = st.absorbed[0];
    m->absorbed[1] = st.absorbed[1];
    m->emitted[0] = st.emitted[0];
    m->emitted[1] = st.emitted[1];
    m->created = st.created;
    m->e_overflow = st.overflow;
    m->see_clamped = st.see_clamped;
    m->n_acc = st.n_acc;
    m->pushed = st.pushed;
    m->volt_amp = st.volt_amp;
    m->p_abs = st.p_abs;
    m->rf_periods = st.rf_periods;
    m->graph_steps = 0;
    m->rollbacks = 0;
    std::vector<int64_t> cnt(nn);
    HD_TRY(hipMemcpy(cnt.data(), d.cnt[st.cbuf], nn * 8, hipMemcpyDeviceToHost));
    int64_t tot = 0;
    for (int j = 0; j < nn; ++j) tot += cnt[j];
    m->n_live = tot >> 32;
    auto sc = [&](int j) { return (j == 0 || j == d.nc) ? h.scale_wall : h.scale_in; };
    if (m->cnt) std::copy(cnt.begin(), cnt.end(), m->cnt);
    if (m->n_e)
      for (int j = 0; j < nn; ++j) m->n_e[j] = (double)cnt[j] * sc(j);
    // ion charge density and flux: species 0 alone, or sum_s Z_s x_s
    const int S = d.S;
    auto net = [&](const double* src, double* out) -> int {
      std::vector<double> a((size_t)S * nn);
      HD_TRY(hipMemcpy(a.data(), src, a.size() * 8, hipMemcpyDeviceToHost));
      for (int j = 0; j < nn; ++j) {
        double v = (double)d.Z[0] * a[j];
        for (int q = 1; q < S; ++q) v = v + (double)d.Z[q] * a[(size_t)q * nn + j];
        out[j] = v;
      }
      return HD_OK;
    };
    if (m->n_i) {
      if (S == 1) HD_TRY(hipMemcpy(m->n_i, d.ni, nn * 8, hipMemcpyDeviceToHost));
      else if (int r = net(d.ni, m->n_i)) return r;
    }
    if (m->gamma_i) {
      if (S == 1) HD_TRY(hipMemcpy(m->gamma_i, d.gam, nn * 8, hipMemcpyDeviceToHost));
      else if (int r = net(d.gam, m->gamma_i)) return r;
    }
    if (m->n_species)
      HD_TRY(hipMemcpy(m->n_species, d.ni, (size_t)S * nn * 8, hipMemcpyDeviceToHost));
    if (m->gamma_species)
      HD_TRY(hipMemcpy(m->gamma_species, d.gam, (size_t)S * nn * 8, hipMemcpyDeviceToHost));
    if (m->phi) HD_TRY(hipMemcpy(m->phi, d.phi, nn * 8, hipMemcpyDeviceToHost));
    if (m->E) HD_TRY(hipMemcpy(m->E, d.E, nn * 8, hipMemcpyDeviceToHost));
    if (m->n_e_avg) {
      std::vector<uint64_t> a(nn);
      HD_TRY(hipMemcpy(a.data(), d.acc_cnt, nn * 8, hipMemcpyDeviceToHost));
      for (int j = 0; j < nn; ++j)
        m->n_e_avg[j] = st.n_acc ? (double)a[j] * sc(j) / (double)st.n_acc : 0.0;
    }
    if (m->n_i_avg) {
      std::vector<double> a(nn);
      HD_TRY(hipMemcpy(a.data(), d.acc_ni, nn * 8, hipMemcpyDeviceToHost));
      for (int j = 0; j < nn; ++j) m->n_i_avg[j] = st.n_acc ? a[j] / (double)st.n_acc : 0.0;
    }
    if (m->eedf_counts || m->eedf) {
      std::vector<uint64_t> e(d.nbins + 1);
      HD_TRY(hipMemcpy(e.data(), d.eedf, e.size() * 8, hipMemcpyDeviceToHost));
      if (m->eedf_counts) std::copy(e.begin(), e.end(), m->eedf_counts);
      if (m->eedf) {
        uint64_t in = 0;
        for (int b = 0; b < d.nbins; ++b) in += e[b];
        const double de = 1.0 / h.keedf;
        for (int b = 0; b < d.nbins; ++b) m->eedf[b] = in ? (double)e[b] / ((double)in * de) : 0.0;
      }
    }
    return rc;
  }

  int particles(int i, int32_t* cell, void* off, void* vx, void* vy, void* vz, uint32_t* id,
                int64_t cap, int64_t* n_out) {
    if (i < 0 || i >= D) return fail(HD_EINVAL, "bad index");
    State st;
    int rc = sync_state(i, st);
    const Disch<P>& d = hs[i].dd;
    const size_t n = st.n_main;
    if (n_out) *n_out = (int64_t)n;
    if (cap < (int64_t)n) return fail(HD_EINVAL, "cap < n_slots");
    const int b = st.buf;
    if (cell) HD_TRY(hipMemcpy(cell, d.cell[b], n * 4, hipMemcpyDeviceToHost));
    if (off) HD_TRY(hipMemcpy(off, d.off[b], n * sizeof(P), hipMemcpyDeviceToHost));
    if (vx) HD_TRY(hipMemcpy(vx, d.vx[b], n * sizeof(P), hipMemcpyDeviceToHost));
    if (vy) HD_TRY(hipMemcpy(vy, d.vy[b], n * sizeof(P), hipMemcpyDeviceToHost));
    if (vz) HD_TRY(hipMemcpy(vz, d.vz[b], n * sizeof(P), hipMemcpyDeviceToHost));
    if (id) HD_TRY(hipMemcpy(id, d.id[b], n * 4, hipMemcpyDeviceToHost));
    return rc;
  }

  // Real steps, one kernel group at a time, with event pairs around each.
  int profile(int64_t n, double* out_ms) {
    if (n <= 0 || !out_ms) return fail(HD_EINVAL, "n_steps must be positive");
    if (error) return fail(error, "handle is in an error state");
    int rc = ensure_volt(host_step + n + 1);
    if (rc) return rc;
    HD_TRY(launch_set_steps<P>(d_desc, D, n, stream));
    std::vector<hipEvent_t> ev((size_t)n * 8);
    for (auto& e : ev) HD_TRY(hipEventCreate(&e));
    std::vector<int> sorted((size_t)n, 0);
    hipError_t err = hipSuccess;
    for (int64_t s = 0; s < n && err == hipSuccess; ++s) {
      hipEvent_t* e = &ev[(size_t)s * 8];
      const bool srt = ((host_step + 1) % sort_every) == 0;
      sorted[(size_t)s] = srt;
      if (host_step % sort_every == 0)
        err = launch_checkpoint<P>(d_desc, D, 0, std::max(1, cus * 2), stream);
      if (err == hipSuccess) err = hipEventRecord(e[0], stream);
      if (err == hipSuccess)
        err = launch_electron_impl<P>(d_desc, D, grid_e, tab_max, nn_max, nb1_max, fluid_nn,
                                      K_max, elec_variant, stream);
      if (err == hipSuccess) err = hipEventRecord(e[1], stream);
      if (err == hipSuccess) err = hipEventRecord(e[2], stream);
      if (err == hipSuccess) err = launch_finalize<P>(d_desc, D, 0, nn_max, grid_a, stream);
      if (err == hipSuccess) err = hipEventRecord(e[3], stream);
      // the append runs inside the end-of-step launch: its slot reads ~0
      if (err == hipSuccess) err = hipEventRecord(e[4], stream);
      if (err == hipSuccess) err = hipEventRecord(e[5], stream);
      if (err == hipSuccess) err = hipEventRecord(e[6], stream);
      if (err == hipSuccess && srt)
        err = launch_sort_impl<P>(d_desc, D, grid_s, tile_s, nc_max, stream);
      if (err == hipSuccess) err = hipEventRecord(e[7], stream);
      host_step += 1;
    }
    if (err == hipSuccess) err = hipStreamSynchronize(stream);
    double acc[5] = {0, 0, 0, 0, 0};
    int nsort = 0;
    for (int64_t s = 0; s < n && err == hipSuccess; ++s) {
      hipEvent_t* e = &ev[(size_t)s * 8];
      float t[5];
      err = hipEventElapsedTime(&t[0], e[0], e[1]);
      if (err == hipSuccess) err = hipEventElapsedTime(&t[1], e[2], e[3]);
      if (err == hipSuccess) err = hipEventElapsedTime(&t[2], e[4], e[5]);
      if (err == hipSuccess) err = hipEventElapsedTime(&t[3], e[6], e[7]);
      if (err == hipSuccess) err = hipEventElapsedTime(&t[4], e[0], e[7]);
      for (int k = 0; k < 5; ++k)
        if (k != 3) acc[k] += t[k];
      if (sorted[(size_t)s]) {
        acc[3] += t[3];
        nsort += 1;
      }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (err != hipSuccess) return fail(HD_EDEVICE, hipGetErrorString(err));
    for (int k = 0; k < 5; ++k) out_ms[k] = k == 3 ? (nsort ? acc[3] / nsort : 0.0) : acc[k] / n;
    return HD_OK;
  }

  // The autotuner (see hd_batch_autotune).  Steps are real steps of the run,
  // launched one kernel at a time with the candidates taken in turn.
  int autotune(int64_t max_steps, hd_launch_config* out) {
    if (error) return fail(error, "handle is in an error state");
    const int64_t n = max_steps / sort_every * sort_every;
    if (n < 2 * (int64_t)sort_every) return fail(HD_EINVAL, "max_steps below two sort intervals");
    int rc = ensure_volt(host_step + n + 1);
    if (rc) return rc;
    struct Cand {
      hd_launch_config c;
      double ms = 0.0;
      int runs = 0;
    };
    std::vector<Cand> ce, cs, ca;  // electron, sort, append candidates
    for (int v = 0; v < electron_variants(); ++v) {
      const int occ = electron_occupancy<P>(tab_max, nn_max, nb1_max, fluid_nn, K_max, D, v);
      if (occ < 1) continue;
      // wide workgroups where the narrow ones fit once per CU or the
      // particle state streams from HBM (measured faster in both cases, and
      // slower where two narrow workgroups per CU work in the MALL), and
      // only as many as fit at once (fewer would leave CUs idle)
      if (v >= kElecWide && state_bytes <= kMallBytes &&
          electron_occupancy<P>(tab_max, nn_max, nb1_max, fluid_nn, K_max, D, v - kElecWide) != 1)
        continue;
      const int full = std::min(cus * occ, (int)kMaxSegs);
      for (int g : {full, std::max(1, full * 3 / 4), std::max(1, full / 2)}) {
        if (v >= kElecWide && g != full) continue;
        hd_launch_config c = launch;
        c.electron_variant = v;
        c.electron_groups = g;
        ce.push_back({c});
      }
    }
    // sort: workgroups at the default tile, then the larger tile (half as
    // many (cell, tile) entries to scan)
    for (int f : {2, 4, 8}) {
      hd_launch_config c = launch;
      c.sort_groups = cus * f;
      c.sort_tile = kSortTile;
      cs.push_back({c});
    }
    {
      hd_launch_config c = launch;
      c.sort_groups = cus * 4;
      c.sort_tile = 2 * kSortTile;
      cs.push_back({c});
    }
    for (int f : {8, 4, 2}) {
      hd_launch_config c = launch;
      c.append_groups = std::max(1, cus / f);
      ca.push_back({c});
    }
    const hd_launch_config keep = launch;
    HD_TRY(launch_set_steps<P>(d_desc, D, n, stream));
    std::vector<hipEvent_t> ev((size_t)n * 6);
    for (auto& e : ev) HD_TRY(hipEventCreate(&e));
    std::vector<int> which((size_t)n * 3, -1);
    // Electron candidates run in blocks of consecutive steps and the first
    // step of a block is not timed: a variant leaves the caches (the MALL
    // above all) in its own state, which the next step inherits.  The other
    // candidates take steps (append) and sorts (sort) in turn.
    const int64_t nce = (int64_t)ce.size();
    const int64_t blk = std::max<int64_t>(2, n / nce);
    hipError_t err = hipSuccess;
    int nsort = 0;
    for (int64_t s = 0; s < n && err == hipSuccess; ++s) {
      hipEvent_t* e = &ev[(size_t)s * 6];
      const bool srt = ((host_step + 1) % sort_every) == 0;
      const int ie = (int)std::min<int64_t>(s / blk, nce - 1);
      const int ia = (int)(s % (int64_t)ca.size());
      const int is = srt ? nsort++ % (int)cs.size() : -1;
      which[(size_t)s * 3] = ie;
      which[(size_t)s * 3 + 1] = ia;
      which[(size_t)s * 3 + 2] = is;
      const int ge = D + ce[ie].c.electron_groups;
      if (host_step % sort_every == 0)
        err = launch_checkpoint<P>(d_desc, D, 0, std::max(1, cus * 2), stream);
      if (err == hipSuccess) err = hipEventRecord(e[0], stream);
      if (err == hipSuccess)
        err = launch_electron_impl<P>(d_desc, D, ge, tab_max, nn_max, nb1_max, fluid_nn, K_max,
                                      ce[ie].c.electron_variant, stream);
      if (err == hipSuccess) err = hipEventRecord(e[1], stream);
      if (err == hipSuccess) err = hipEventRecord(e[2], stream);
      if (err == hipSuccess)
        err = launch_finalize<P>(d_desc, D, 0, nn_max, ca[ia].c.append_groups, stream);
      if (err == hipSuccess) err = hipEventRecord(e[3], stream);
      if (err == hipSuccess) err = hipEventRecord(e[4], stream);
      if (err == hipSuccess && srt)
        err = launch_sort_impl<P>(d_desc, D, cs[is].c.sort_groups, cs[is].c.sort_tile, nc_max,
                                  stream);
      if (err == hipSuccess) err = hipEventRecord(e[5], stream);
      host_step += 1;
    }
    if (err == hipSuccess) err = hipStreamSynchronize(stream);
    for (int64_t s = 0; s < n && err == hipSuccess; ++s) {
      hipEvent_t* e = &ev[(size_t)s * 6];
      float t0 = 0, t1 = 0, t2 = 0;
      err = hipEventElapsedTime(&t0, e[0], e[1]);
      if (err == hipSuccess) err = hipEventElapsedTime(&t1, e[2], e[3]);
      if (err == hipSuccess) err = hipEventElapsedTime(&t2, e[4], e[5]);
      if (err != hipSuccess) break;
      if (s % blk != 0) {
        Cand& a = ce[which[(size_t)s * 3]];
        a.ms += t0;
        a.runs += 1;
      }
      Cand& b = ca[which[(size_t)s * 3 + 1]];
      b.ms += t1;
      b.runs += 1;
      if (which[(size_t)s * 3 + 2] >= 0) {
        Cand& c = cs[which[(size_t)s * 3 + 2]];
        c.ms += t2;
        c.runs += 1;
      }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (err != hipSuccess) return fail(HD_EDEVICE, hipGetErrorString(err));
    auto best = [](const std::vector<Cand>& v) {
      size_t b = 0;
      double bm = 1e300;
      for (size_t i = 0; i < v.size(); ++i)
        if (v[i].runs && v[i].ms / v[i].runs < bm) {
          bm = v[i].ms / v[i].runs;
          b = i;
        }
      return v[b].c;
    };
    hd_launch_config c = keep;
    const hd_launch_config be = best(ce), bs = best(cs), ba = best(ca);
    c.electron_variant = be.electron_variant;
    c.electron_groups = be.electron_groups;
    c.sort_groups = bs.sort_groups;
    c.sort_tile = bs.sort_tile;
    c.append_groups = ba.append_groups;
    rc = apply_launch(c);
    if (rc) return rc;
    tune_store(tune_key, launch);
    if (out) *out = launch;
    return HD_OK;
  }

  int push_field(int i, void* out) {
    State st;
    int rc = sync_state(i, st);
    HD_TRY(hipMemcpy(out, hs[i].dd.Ep, hs[i].dd.nn * sizeof(P), hipMemcpyDeviceToHost));
    return rc;
  }
};

template <class P>
size_t required_bytes(const hd_params& p) {
  return layout<P>(p, kVoltInitial).total + sizeof(Disch<P>);
}

// ---------------------------------------------------------------------------
// Served job stream: continuous batching over a fixed set of slots.  A host
// thread admits queued jobs into free slots while the device-memory budget
// allows, replays one captured interval of sort_every steps over all slots
// (idle slots point at an idle State and cost nothing), and retires jobs that
// reached their step count.  Jobs start at interval boundaries, so each
// job's steps -- and its result -- are exactly those of a run alone.
// ---------------------------------------------------------------------------
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct JobResult {
  std::vector<double> n_e, n_i, phi, E, gam, n_e_avg, n_i_avg, eedf;
  std::vector<int64_t> cnt;
  std::vector<uint64_t> eedf_counts;
  hd_moment_set m{};
};

struct Job {
  uint64_t id = 0;
  hd_params p{};
  std::vector<hd_xs_channel> ch;
  std::vector<std::vector<double>> sig;
  int64_t n_steps = 0;
  size_t bytes = 0;
  int state = 0;  // 0 queued, 1 running, 2 done, 3 failed
  int err = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  JobResult res;
  int prep_state = 0;           // host preparation: 0 not started, 1 running, 2 done
  std::shared_ptr<void> prep;   // the prepared host state (the server's type)
  std::atomic<bool> cancel{false};  // running job to retire after the interval in flight
};

struct ServerBase {
  virtual ~ServerBase() {}
  virtual int submit(const hd_params* p, int64_t n, uint64_t* id) = 0;
  virtual int poll(uint64_t id, int32_t* state, hd_moment_set* out, double* times) = 0;
  virtual int stats(hd_server_counters* out) = 0;
  virtual int drain(double timeout_s) = 0;
  virtual int cancel(uint64_t id) = 0;
};

template <class P>
struct Server : ServerBase {
  using B = Batch<P>;
  hd_server_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr, own_stream = nullptr;
  int S = 0;
  Disch<P>* d_desc = nullptr;
  State* d_idle = nullptr;
  DevMem mem;  // the admitted jobs' blocks (hipMalloc; released when a job retires)
  std::vector<Host<P>> hs;
  std::vector<Job*> slot_job;
  std::vector<int64_t> slot_done;  // steps completed by the job in the slot
  int grid_e = 0, grid_a = 0, grid_s = 0, tab_max = 0, nn_max = 0, nb1_max = 0, nc_max = 0,
      fluid_nn = 0, K_max = 1;
  // One interval over all slots, captured twice: with the default electron
  // variant, and with nontemporal traffic of ids, cells and offsets for when
  // the admitted jobs' particle state is larger than the MALL (results are
  // the same).
  hipGraphExec_t graph = nullptr, graph_nt = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  int worker_err = 0;
  std::string worker_msg;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::deque<Job*> queue;
  uint64_t next_job = 1;
  size_t used = 0;
  uint64_t chunks = 0, pushed_done = 0, completed = 0, failed = 0, cancelled = 0;
  double busy_s = 0, t_start = 0;

  // A job's host-side state, prepared ahead of admission.
  struct Prep {
    Host<P> h;
    typename B::Prepared pr;
  };
  static constexpr size_t kPrepAhead = 32;  // queued jobs prepared ahead at most
  std::vector<std::thread> preppers;
  bool stop_prep = false;

  ~Server() override {
    {
      std::lock_guard<std::mutex> g(mu);
      stop = true;
    }
    cv.notify_all();
    if (worker.joinable()) worker.join();
    {
      std::lock_guard<std::mutex> g(mu);
      stop_prep = true;
    }
    cv.notify_all();
    for (auto& t : preppers)
      if (t.joinable()) t.join();
    if (graph) (void)hipGraphExecDestroy(graph);
    if (graph_nt) (void)hipGraphExecDestroy(graph_nt);
    for (auto& h : hs)
      if (h.base) mem.release(h.base);
    if (d_desc) (void)hipFree(d_desc);
    if (d_idle) (void)hipFree(d_idle);
    if (own_stream) (void)hipStreamDestroy(own_stream);
  }

  // An empty slot: no cells, no particles, its own idle state.
  Disch<P> idle_entry(int slot) const {
    Disch<P> e{};
    e.st = d_idle + slot;
    e.sort_every = 1;  // never used (the state is idle), but no interval is 0
    e.eedf_every = 1;
    return e;
  }

  int create(const hd_server_config* c, const hd_device_ctx* ctx) {
    if (ctx && ctx->arena) return fail(HD_EINVAL, "the server takes no arena");
    cfg = *c;
    S = cfg.max_slots;
    device = ctx ? ctx->device : 0;
    stream = ctx ? (hipStream_t)ctx->stream : nullptr;
    HD_TRY(hipSetDevice(device));
    if (!stream) {
      HD_TRY(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
      stream = own_stream;
    }
    tab_max = cfg.max_energy * std::max(1, cfg.max_channels);
    K_max = std::max(1, cfg.max_channels);
    nn_max = cfg.max_cells + 1;
    nc_max = cfg.max_cells;
    nb1_max = cfg.max_eedf_bins + 1;
    fluid_nn = cfg.allow_full_fluid ? nn_max : 0;
    hipDeviceProp_t prop;
    HD_TRY(hipGetDeviceProperties(&prop, device));
    const size_t lds = electron_lds_bytes<P>(S, tab_max, nn_max, nb1_max, fluid_nn, K_max, 0);
    if (lds > (size_t)prop.sharedMemPerBlock) return fail(HD_EINVAL, "slot caps exceed LDS");
    HD_TRY(sort_set_lds<P>(nc_max, S));
    HD_TRY(finalize_set_lds<P>(nn_max));
    const int occ = electron_occupancy<P>(tab_max, nn_max, nb1_max, fluid_nn, K_max, S, 0);
    if (occ < 1) return fail(HD_EDEVICE, "electron kernel cannot be resident");
    const int v_plain = widen_variant<P>(0, tab_max, nn_max, nb1_max, fluid_nn, K_max, S);
    const int v_stream =
        widen_variant<P>(kElecVariantStreaming, tab_max, nn_max, nb1_max, fluid_nn, K_max, S);
    grid_e = S + std::min(prop.multiProcessorCount * occ, (int)kMaxSegs);
    grid_a = std::max(1, prop.multiProcessorCount / 4);
    grid_s = prop.multiProcessorCount * 4;
    HD_TRY(hipMalloc((void**)&d_idle, sizeof(State) * (size_t)S));
    HD_TRY(hipMemset(d_idle, 0, sizeof(State) * (size_t)S));
    HD_TRY(hipMalloc((void**)&d_desc, sizeof(Disch<P>) * S));
    hs.resize(S);
    slot_job.assign(S, nullptr);
    slot_done.assign(S, 0);
    std::vector<Disch<P>> v;
    for (int i = 0; i < S; ++i) v.push_back(idle_entry(i));
    HD_TRY(hipMemcpy(d_desc, v.data(), sizeof(Disch<P>) * S, hipMemcpyHostToDevice));
    // capture one interval of sort_every steps over all slots, per variant
    for (int nt = 0; nt < 2; ++nt) {
      hipGraph_t g = nullptr;
      HD_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      for (int s = 0; s < cfg.sort_every && e == hipSuccess; ++s) {
        e = launch_electron_impl<P>(d_desc, S, grid_e, tab_max, nn_max, nb1_max, fluid_nn, K_max,
                                    nt ? v_stream : v_plain, stream);
        if (e == hipSuccess) e = launch_finalize<P>(d_desc, S, 0, nn_max, grid_a, stream);
        if (e == hipSuccess && s == cfg.sort_every - 1)
          e = launch_sort_impl<P>(d_desc, S, grid_s, kSortTile, nc_max, stream);
      }
      const hipError_t e2 = hipStreamEndCapture(stream, &g);
      if (e != hipSuccess || e2 != hipSuccess)
        return fail(HD_EDEVICE, std::string("capture failed: ") + hipGetErrorString(e ? e : e2));
      e = hipGraphInstantiate(nt ? &graph_nt : &graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(HD_EDEVICE, hipGetErrorString(e));
    }
    t_start = now_s();
    worker = std::thread([this]() { loop(); });
    const unsigned hc = std::thread::hardware_concurrency();
    const int np = (int)std::min(16u, std::max(2u, hc / 2));
    for (int t = 0; t < np; ++t) preppers.emplace_back([this]() { prep_loop(); });
    return HD_OK;
  }

  // Host-side preparation of queued jobs (tables, initial load, drive table)
  // ahead of admission, on threads of their own, so that admitting a job
  // only uploads it; the first kPrepAhead queued jobs in order.
  void prep_loop() {
    for (;;) {
      Job* j = nullptr;
      {
        std::unique_lock<std::mutex> g(mu);
        for (;;) {
          if (stop_prep) return;
          size_t k = 0;
          for (Job* q : queue) {
            if (k++ >= kPrepAhead) break;
            if (q->prep_state == 0) {
              j = q;
              break;
            }
          }
          if (j) break;
          cv.wait_for(g, std::chrono::milliseconds(5));
        }
        j->prep_state = 1;
      }
      auto pp = std::make_shared<Prep>();
      pp->h.p = j->p;
      pp->h.p.channels = j->ch.empty() ? nullptr : j->ch.data();
      B::prepare_host(pp->h, std::max<int64_t>(kVoltInitial, j->n_steps + 2), pp->pr);
      {
        std::lock_guard<std::mutex> g(mu);
        j->prep = pp;
        j->prep_state = 2;
      }
      cv.notify_all();
    }
  }

  int submit(const hd_params* p, int64_t n, uint64_t* id) override {
    std::string why;
    if (!validate(p, why)) return fail(HD_EINVAL, why);
    if (n < 1) return fail(HD_EINVAL, "n_steps must be positive");
    if (p->precision != cfg.precision || p->sort_every != cfg.sort_every ||
        p->eedf_every != cfg.eedf_every || p->n_cells > cfg.max_cells ||
        p->n_energy > cfg.max_energy || p->n_channels > cfg.max_channels ||
        p->n_energy * std::max(1, p->n_channels) > tab_max ||
        p->n_eedf_bins > cfg.max_eedf_bins ||
        (full_fluid(p->ion_model) && !cfg.allow_full_fluid) ||
        p->ion_model == HD_ION_DD_SPECIES)
      return fail(HD_EINVAL, "job does not fit the server's slot configuration");
    auto job = std::make_unique<Job>();
    job->p = *p;
    job->sig.resize(p->n_channels);
    job->ch.resize(p->n_channels);
    for (int k = 0; k < p->n_channels; ++k) {
      job->sig[k].assign(p->channels[k].sigma_m2, p->channels[k].sigma_m2 + p->n_energy);
      job->ch[k] = p->channels[k];
      job->ch[k].sigma_m2 = job->sig[k].data();
    }
    job->p.channels = job->ch.empty() ? nullptr : job->ch.data();
    job->n_steps = n;
    job->bytes = layout<P>(job->p, std::max<int64_t>(kVoltInitial, n + 2)).total;
    if (job->bytes > cfg.hbm_budget_bytes) return fail(HD_ENOMEM, "job exceeds the HBM budget");
    job->t_submit = now_s();
    std::lock_guard<std::mutex> g(mu);
    if (worker_err) return fail(worker_err, worker_msg);
    job->id = next_job++;
    *id = job->id;
    queue.push_back(job.get());
    jobs[job->id] = std::move(job);
    cv.notify_all();
    return HD_OK;
  }

  void set_error(int code, const std::string& m) {
    std::lock_guard<std::mutex> g(mu);
    worker_err = code;
    worker_msg = m;
    stop = true;
    cv.notify_all();
  }

  // Admit one job into a slot (worker thread; device calls on the stream).
  int admit(int slot, Job* job) {
    std::shared_ptr<Prep> pp;
    {
      std::lock_guard<std::mutex> g(mu);
      pp = std::static_pointer_cast<Prep>(job->prep);
      job->prep.reset();
    }
    Host<P>& h = hs[slot];
    h = std::move(pp->h);
    int rc = B::upload_state(h, pp->pr, stream, mem);
    pp.reset();
    if (rc) return rc;
    HD_TRY(hipMemcpyAsync(d_desc + slot, &h.dd, sizeof(Disch<P>), hipMemcpyHostToDevice, stream));
    HD_TRY(launch_finalize<P>(d_desc + slot, 1, 1, nn_max, 0, stream));
    const int64_t n = job->n_steps;
    HD_TRY(hipMemcpyAsync(&h.dd.st->steps_left, &n, sizeof(int64_t), hipMemcpyHostToDevice,
                          stream));
    HD_TRY(hipStreamSynchronize(stream));
    slot_job[slot] = job;
    slot_done[slot] = 0;
    return HD_OK;
  }

  int retire(int slot) {
    Host<P>& h = hs[slot];
    Job* job = slot_job[slot];
    State st;
    HD_TRY(hipMemcpy(&st, h.dd.st, sizeof(State), hipMemcpyDeviceToHost));
    const int nn = h.dd.nn;
    JobResult& r = job->res;
    r.n_e.resize(nn);
    r.n_i.resize(nn);
    r.phi.resize(nn);
    r.E.resize(nn);
    r.gam.resize(nn);
    r.n_e_avg.resize(nn);
    r.n_i_avg.resize(nn);
    r.cnt.resize(nn);
    r.eedf_counts.resize(h.dd.nbins + 1);
    r.eedf.resize(h.dd.nbins);
    hd_moment_set& m = r.m;
    m.n_e = r.n_e.data();
    m.n_i = r.n_i.data();
    m.phi = r.phi.data();
    m.E = r.E.data();
    m.gamma_i = r.gam.data();
    m.n_e_avg = r.n_e_avg.data();
    m.n_i_avg = r.n_i_avg.data();
    m.cnt = r.cnt.data();
    m.eedf_counts = r.eedf_counts.data();
    m.eedf = r.eedf.data();
    const int rc = B::fill_moments(h, st, &m);
    const Disch<P> ie = idle_entry(slot);
    HD_TRY(hipMemcpy(d_desc + slot, &ie, sizeof(Disch<P>), hipMemcpyHostToDevice));
    mem.release(h.base);
    h.base = nullptr;
    std::lock_guard<std::mutex> g(mu);
    job->t_done = now_s();
    job->err = st.error ? st.error : rc;
    if (job->cancel) {
      job->state = 4;
      cancelled += 1;
    } else {
      job->state = job->err ? 3 : 2;
      (job->err ? failed : completed) += 1;
    }
    pushed_done += st.pushed;
    used -= job->bytes;
    slot_job[slot] = nullptr;
    cv.notify_all();
    return HD_OK;
  }

  void loop() {
    if (hipSetDevice(device) != hipSuccess) return set_error(HD_EDEVICE, "hipSetDevice failed");
    for (;;) {
      std::vector<std::pair<int, Job*>> admits;
      {
        std::unique_lock<std::mutex> g(mu);
        for (int s = 0; s < S && !queue.empty(); ++s) {
          if (slot_job[s]) continue;
          Job* j = queue.front();
          if (j->prep_state != 2) break;  // first come, first admitted: wait for its host state
          if (used + j->bytes > cfg.hbm_budget_bytes) break;
          queue.pop_front();
          used += j->bytes;
          j->state = 1;
          j->t_admit = now_s();
          slot_job[s] = j;  // reserved
          admits.push_back({s, j});
        }
        bool active = !admits.empty();
        for (int s = 0; s < S; ++s) active = active || slot_job[s] != nullptr;
        if (!active) {
          if (stop) return;
          cv.wait_for(g, std::chrono::milliseconds(2));
          continue;
        }
      }
      for (auto& a : admits) {
        const int rc = admit(a.first, a.second);
        if (rc) return set_error(rc, g_err);
      }
      // particle bytes of the admitted jobs (their initial loads): beyond the
      // MALL the interval runs the streaming electron variant
      uint64_t resident = 0;
      for (int s = 0; s < S; ++s)
        if (slot_job[s]) resident += (uint64_t)slot_job[s]->p.n_macro * (8u + 4u * sizeof(P));
      hipGraphExec_t run = resident > kMallBytes ? graph_nt : graph;
      const double t0 = now_s();
      if (hipGraphLaunch(run, stream) != hipSuccess || hipStreamSynchronize(stream) != hipSuccess)
        return set_error(HD_EDEVICE, "interval launch failed");
      busy_s += now_s() - t0;
      chunks += 1;
      for (int s = 0; s < S; ++s) {
        Job* j = slot_job[s];
        if (!j) continue;
        slot_done[s] += cfg.sort_every;
        if (slot_done[s] >= j->n_steps || j->cancel) {
          const int rc = retire(s);
          if (rc) return set_error(rc, g_err);
        }
      }
      std::lock_guard<std::mutex> g(mu);
      if (stop && queue.empty()) {
        bool active = false;
        for (int s = 0; s < S; ++s) active = active || slot_job[s] != nullptr;
        if (!active) return;
      }
    }
  }

  int poll(uint64_t id, int32_t* state, hd_moment_set* out, double* times) override {
    std::lock_guard<std::mutex> g(mu);
    auto it = jobs.find(id);
    if (it == jobs.end()) return fail(HD_EINVAL, "unknown job");
    Job* j = it->second.get();
    if (state) *state = j->state;
    if (times) {
      times[0] = j->state >= 1 ? j->t_admit - j->t_submit : -1.0;
      times[1] = j->state >= 2 ? j->t_done - j->t_submit : -1.0;
      times[2] = j->state >= 2 ? j->t_done - j->t_admit : -1.0;
    }
    if (j->state < 2 || j->state == 4 || !out) return HD_OK;  // no result (yet)
    const hd_moment_set& m = j->res.m;
    double* arr_out[] = {out->n_e, out->n_i, out->phi, out->E, out->gamma_i, out->n_e_avg,
                         out->n_i_avg};
    const double* arr_in[] = {m.n_e, m.n_i, m.phi, m.E, m.gamma_i, m.n_e_avg, m.n_i_avg};
    for (int k = 0; k < 7; ++k)
      if (arr_out[k]) std::copy(arr_in[k], arr_in[k] + m.n_nodes, arr_out[k]);
    if (out->cnt) std::copy(m.cnt, m.cnt + m.n_nodes, out->cnt);
    if (out->eedf_counts) std::copy(m.eedf_counts, m.eedf_counts + m.n_eedf_bins + 1, out->eedf_counts);
    if (out->eedf) std::copy(m.eedf, m.eedf + m.n_eedf_bins, out->eedf);
    hd_moment_set keep = *out;
    *out = m;
    out->n_e = keep.n_e;
    out->n_i = keep.n_i;
    out->phi = keep.phi;
    out->E = keep.E;
    out->gamma_i = keep.gamma_i;
    out->n_e_avg = keep.n_e_avg;
    out->n_i_avg = keep.n_i_avg;
    out->cnt = keep.cnt;
    out->eedf_counts = keep.eedf_counts;
    out->eedf = keep.eedf;
    return j->err ? fail(j->err, "job failed on the device") : HD_OK;
  }

  int stats(hd_server_counters* out) override {
    std::lock_guard<std::mutex> g(mu);
    out->submitted = next_job - 1;
    out->completed = completed;
    out->failed = failed;
    out->queued = queue.size();
    uint64_t running = 0;
    for (int s = 0; s < S; ++s) running += slot_job[s] ? 1 : 0;
    out->running = running;
    out->intervals = chunks;
    out->particle_steps = pushed_done;
    out->bytes_in_use = used;
    out->busy_s = busy_s;
    out->wall_s = now_s() - t_start;
    out->error = worker_err;
    out->cancelled = (int32_t)cancelled;
    return worker_err ? fail(worker_err, worker_msg) : HD_OK;
  }

  // A queued job leaves the queue at once; a running one is retired after
  // the interval in flight (its slot and bytes freed, no result kept).
  int cancel(uint64_t id) override {
    std::lock_guard<std::mutex> g(mu);
    auto it = jobs.find(id);
    if (it == jobs.end()) return fail(HD_EINVAL, "unknown job");
    Job* j = it->second.get();
    if (j->state == 0) {
      auto q = std::find(queue.begin(), queue.end(), j);
      if (q != queue.end()) queue.erase(q);
      j->state = 4;
      j->t_done = now_s();
      cancelled += 1;
      cv.notify_all();
    } else if (j->state == 1) {
      j->cancel = true;
    }
    return HD_OK;
  }

  int drain(double timeout_s) override {
    const double t_end = now_s() + timeout_s;
    std::unique_lock<std::mutex> g(mu);
    for (;;) {
      if (worker_err) return fail(worker_err, worker_msg);
      bool busy = !queue.empty();
      for (int s = 0; s < S; ++s) busy = busy || slot_job[s] != nullptr;
      if (!busy) return HD_OK;
      if (now_s() > t_end) return fail(HD_ESTATE, "drain timed out");
      cv.wait_for(g, std::chrono::milliseconds(5));
    }
  }
};


// ---------------------------------------------------------------------------
// Auxiliary ion swarm (Sec. II.C).
// ---------------------------------------------------------------------------
struct SwarmBase {
  virtual ~SwarmBase() {}
  virtual int run(int64_t n, int accumulate) = 0;
  virtual int results(hd_swarm_result* out) = 0;
  virtual int ions(int f, void* vx, void* vy, void* vz, double* avz, double* av2, int64_t cap) = 0;
};

namespace {

bool swarm_valid(const hd_swarm_params* p, std::string& why) {
  if (!p) return (why = "null params"), false;
  if (p->abi_version != HD_ABI_VERSION) return (why = "abi_version mismatch"), false;
  if (p->precision != HD_FP32 && p->precision != HD_FP64) return (why = "precision"), false;
  if (p->n_fields < 1 || p->n_ions < 1 || (int64_t)p->n_fields * p->n_ions > ((int64_t)1 << 31) ||
      p->n_ions > ((int64_t)1 << 32) - 1)
    return (why = "n_fields * n_ions must lie in [1, 2^31]"), false;
  if (p->n_energy < 2 || p->n_energy > kSwarmMaxEnergy)
    return (why = "n_energy out of [2, 4096]"), false;
  if (!p->rate_m3_s || !p->e0_V_m) return (why = "rate table or field list missing"), false;
  for (int i = 0; i < p->n_energy; ++i)
    if (!(p->rate_m3_s[i] >= 0) || !std::isfinite(p->rate_m3_s[i]))
      return (why = "rate coefficients must be finite and non-negative"), false;
  for (int f = 0; f < p->n_fields; ++f)
    if (!std::isfinite(p->e0_V_m[f])) return (why = "fields must be finite"), false;
  if (!(p->dt_s > 0) || !(p->inv_de_per_eV > 0) || !(p->m_ion_amu > 0) || !(p->m_gas_amu > 0) ||
      !(p->n_gas_m3 >= 0) || !(p->t_gas_K >= 0) || !(p->t_i0_K >= 0))
    return (why = "gas, mass, time step or energy grid"), false;
  return true;
}

// The swarm's constants from its parameters: the same formulas as the
// oracle, FP64 then rounded to P.  Fills w's scalars, the rate table
// tab[n_energy] = P_max nu_i / nu_max and the velocity gain acc[n_fields]
// = e E0 dt / M; returns M.
template <class P>
double swarm_constants(const hd_swarm_params& p, SwarmDev<P>& w, P* tab, P* acc) {
  const int ne = p.n_energy, D = p.n_fields;
  const double M = p.m_ion_amu * kAmu;
  const double MN = p.m_gas_amu * kAmu;
  const double Mr = (M * MN) / (M + MN);
  double nu_max = 0.0;
  for (int i = 0; i < ne; ++i) {
    const double nu = p.n_gas_m3 * p.rate_m3_s[i];
    if (nu > nu_max) nu_max = nu;
  }
  const double Pmax = 1.0 - std::exp(-nu_max * p.dt_s);
  for (int i = 0; i < ne; ++i) {
    const double nu = p.n_gas_m3 * p.rate_m3_s[i];
    tab[i] = (P)(nu_max > 0 ? Pmax * (nu / nu_max) : 0.0);
  }
  for (int f = 0; f < D; ++f) acc[f] = (P)(((kE * p.e0_V_m[f]) * p.dt_s) / M);
  w.n_fields = D;
  w.ne = ne;
  w.n_ions = p.n_ions;
  w.seed = p.seed;
  w.Pmax = (P)Pmax;
  w.KEr = (P)(Mr / (2.0 * kE));
  w.inv_dE = (P)p.inv_de_per_eV;
  w.m1 = (P)(M / (M + MN));
  w.m2 = (P)(MN / (M + MN));
  w.vth_n = std::sqrt(kKb * p.t_gas_K / MN);
  w.vth_i0 = std::sqrt(kKb * p.t_i0_K / M);
  return M;
}

// Results of the swarms from the ion sums over n_acc accumulated steps.
void swarm_fill_results(const hd_swarm_params& p, double M, int64_t n_acc, const double* sums,
                        const uint64_t* coll, const uint64_t* over, hd_swarm_result* out) {
  const int64_t samples = n_acc * p.n_ions;
  for (int f = 0; f < p.n_fields; ++f) {
    const double e0 = p.e0_V_m[f];
    hd_swarm_result& r = out[f];
    r.e0_V_m = e0;
    r.drift_m_s = samples ? sums[2 * f] / (double)samples : 0.0;
    r.mean_energy_eV = samples ? ((0.5 * M) * (sums[2 * f + 1] / (double)samples)) / kE : 0.0;
    r.mobility_m2_Vs = e0 != 0.0 ? r.drift_m_s / e0 : 0.0;
    r.nu_s = r.drift_m_s != 0.0 ? (kE * e0) / (M * r.drift_m_s) : 0.0;
    r.collisions = coll[f];
    r.overflow = over[f];
    r.samples = samples;
  }
}

template <class P>
struct SwarmImpl : SwarmBase {
  hd_swarm_params p{};
  std::vector<double> rate, e0;
  double M = 0;
  hipStream_t stream = nullptr, own_stream = nullptr;
  int device = 0;
  unsigned char* base = nullptr;
  SwarmDev<P> w{};
  int64_t step = 0, n_acc = 0;

  ~SwarmImpl() override {
    if (base) (void)hipFree(base);
    if (own_stream) (void)hipStreamDestroy(own_stream);
  }

  int create(const hd_swarm_params* pp, const hd_device_ctx* ctx) {
    p = *pp;
    rate.assign(pp->rate_m3_s, pp->rate_m3_s + pp->n_energy);
    e0.assign(pp->e0_V_m, pp->e0_V_m + pp->n_fields);
    p.rate_m3_s = rate.data();
    p.e0_V_m = e0.data();
    stream = ctx ? (hipStream_t)ctx->stream : nullptr;
    device = ctx ? ctx->device : 0;
    HD_TRY(hipSetDevice(device));
    if (!stream) {
      HD_TRY(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
      stream = own_stream;
    }
    const int ne = p.n_energy, D = p.n_fields;
    std::vector<P> tab(ne), acc(D);
    M = swarm_constants<P>(p, w, tab.data(), acc.data());
    // one device block: a, tab, vx, vy, vz, avz, av2, coll, over, sums
    const size_t n = (size_t)D * (size_t)p.n_ions;
    size_t off = 0;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off = align_up(off + bytes, 256);
      return o;
    };
    const size_t o_a = take(D * sizeof(P)), o_tab = take(ne * sizeof(P));
    const size_t o_vx = take(n * sizeof(P)), o_vy = take(n * sizeof(P)), o_vz = take(n * sizeof(P));
    const size_t o_az = take(n * 8), o_a2 = take(n * 8);
    const size_t o_c = take(D * 8), o_o = take(D * 8), o_s = take(2 * D * 8);
    if (hipMalloc((void**)&base, off) != hipSuccess) {
      base = nullptr;
      return fail(HD_ENOMEM, "swarm allocation of " + std::to_string(off) + " bytes failed");
    }
    w.a = (const P*)(base + o_a);
    w.tab = (const P*)(base + o_tab);
    w.vx = (P*)(base + o_vx);
    w.vy = (P*)(base + o_vy);
    w.vz = (P*)(base + o_vz);
    w.avz = (double*)(base + o_az);
    w.av2 = (double*)(base + o_a2);
    w.coll = (uint64_t*)(base + o_c);
    w.over = (uint64_t*)(base + o_o);
    w.sums = (double*)(base + o_s);
    HD_TRY(hipMemsetAsync(base + o_c, 0, o_s - o_c + 2 * D * 8, stream));
    HD_TRY(hipMemcpyAsync(base + o_a, acc.data(), D * sizeof(P), hipMemcpyHostToDevice, stream));
    HD_TRY(hipMemcpyAsync(base + o_tab, tab.data(), ne * sizeof(P), hipMemcpyHostToDevice, stream));
    HD_TRY(launch_swarm_init<P>(w, stream));
    HD_TRY(hipStreamSynchronize(stream));
    return HD_OK;
  }

  int run(int64_t n, int accumulate) override {
    if (n < 0) return fail(HD_EINVAL, "n_steps must be non-negative");
    HD_TRY(hipSetDevice(device));
    constexpr int64_t kChunk = 256;  // steps per launch
    for (int64_t done = 0; done < n; done += kChunk) {
      const int k = (int)std::min<int64_t>(kChunk, n - done);
      HD_TRY(launch_swarm_step<P>(w, (uint32_t)(step + done), k, accumulate ? 1 : 0, stream));
    }
    step += n;
    if (accumulate) n_acc += n;
    return HD_OK;
  }

  int results(hd_swarm_result* out) override {
    if (!out) return fail(HD_EINVAL, "null output");
    const int D = p.n_fields;
    HD_TRY(hipSetDevice(device));
    HD_TRY(launch_swarm_reduce<P>(w, stream));
    std::vector<double> sums(2 * D);
    std::vector<uint64_t> coll(D), over(D);
    HD_TRY(hipMemcpyAsync(sums.data(), w.sums, 2 * D * 8, hipMemcpyDeviceToHost, stream));
    HD_TRY(hipMemcpyAsync(coll.data(), w.coll, D * 8, hipMemcpyDeviceToHost, stream));
    HD_TRY(hipMemcpyAsync(over.data(), w.over, D * 8, hipMemcpyDeviceToHost, stream));
    HD_TRY(hipStreamSynchronize(stream));
    swarm_fill_results(p, M, n_acc, sums.data(), coll.data(), over.data(), out);
    return HD_OK;
  }

  int ions(int f, void* vx, void* vy, void* vz, double* avz, double* av2, int64_t cap) override {
    if (f < 0 || f >= p.n_fields) return fail(HD_EINVAL, "field index out of range");
    if (cap < p.n_ions) return fail(HD_EINVAL, "cap < n_ions");
    HD_TRY(hipSetDevice(device));
    const size_t n = (size_t)p.n_ions, o = (size_t)f * n;
    if (vx) HD_TRY(hipMemcpyAsync(vx, w.vx + o, n * sizeof(P), hipMemcpyDeviceToHost, stream));
    if (vy) HD_TRY(hipMemcpyAsync(vy, w.vy + o, n * sizeof(P), hipMemcpyDeviceToHost, stream));
    if (vz) HD_TRY(hipMemcpyAsync(vz, w.vz + o, n * sizeof(P), hipMemcpyDeviceToHost, stream));
    if (avz) HD_TRY(hipMemcpyAsync(avz, w.avz + o, n * 8, hipMemcpyDeviceToHost, stream));
    if (av2) HD_TRY(hipMemcpyAsync(av2, w.av2 + o, n * 8, hipMemcpyDeviceToHost, stream));
    HD_TRY(hipStreamSynchronize(stream));
    return HD_OK;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// The ion swarm for callers that cannot allocate device memory.  Its work
// space is a fixed array in the library's device code, one per device the
// library runs on, held until the process ends.  Host code never takes the
// array's name as an address: each device's address comes from
// hipGetSymbolAddress with that device current, once, and is kept here.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kNoAllocFields = 256;
constexpr int kNoAllocDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocDevices] = {};

// The calling thread's current device must be `device`.
int scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kNoAllocDevices) return fail(HD_EINVAL, "device ordinal");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(HD_EDEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return HD_OK;
}

template <class P>
int swarm_noalloc(const hd_swarm_params& p, int64_t n_relax, int64_t n_avg, hipStream_t stream,
                  int device, hd_swarm_result* out) {
  const int D = p.n_fields, ne = p.n_energy;
  if (D > kNoAllocFields)
    return fail(HD_EINVAL, "more than " + std::to_string(kNoAllocFields) + " fields");
  const size_t n = (size_t)D * (size_t)p.n_ions;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t o_a = take(D * sizeof(P)), o_tab = take(ne * sizeof(P));
  const size_t o_vx = take(n * sizeof(P)), o_vy = take(n * sizeof(P)), o_vz = take(n * sizeof(P));
  const size_t o_az = take(n * 8), o_a2 = take(n * 8);
  const size_t o_c = take(D * 8), o_o = take(D * 8), o_s = take(2 * D * 8);
  if (off > kNoAllocBytes)
    return fail(HD_EINVAL, "the swarm needs " + std::to_string(off) +
                               " bytes of work space; the no-allocation work space holds " +
                               std::to_string(kNoAllocBytes));
  unsigned char* base = nullptr;
  if (int rc = scratch_address(device, &base)) return rc;
  SwarmDev<P> w{};
  P tab[kSwarmMaxEnergy], acc[kNoAllocFields];
  const double M = swarm_constants<P>(p, w, tab, acc);
  w.a = (const P*)(base + o_a);
  w.tab = (const P*)(base + o_tab);
  w.vx = (P*)(base + o_vx);
  w.vy = (P*)(base + o_vy);
  w.vz = (P*)(base + o_vz);
  w.avz = (double*)(base + o_az);
  w.av2 = (double*)(base + o_a2);
  w.coll = (uint64_t*)(base + o_c);
  w.over = (uint64_t*)(base + o_o);
  w.sums = (double*)(base + o_s);
  HD_TRY(hipMemcpyAsync(base + o_a, acc, D * sizeof(P), hipMemcpyHostToDevice, stream));
  HD_TRY(hipMemcpyAsync(base + o_tab, tab, ne * sizeof(P), hipMemcpyHostToDevice, stream));
  // the work space keeps the previous call's contents: counters and sums
  // start at zero, velocities and ion sums are set by the load
  HD_TRY(launch_swarm_clear<P>(w, stream));
  HD_TRY(launch_swarm_init<P>(w, stream));
  constexpr int64_t kChunk = 256;  // steps per launch, as hd_swarm_run
  int64_t step = 0;
  for (int acc_on = 0; acc_on < 2; ++acc_on) {
    const int64_t m = acc_on ? n_avg : n_relax;
    for (int64_t done = 0; done < m; done += kChunk) {
      const int k = (int)std::min<int64_t>(kChunk, m - done);
      HD_TRY(launch_swarm_step<P>(w, (uint32_t)(step + done), k, acc_on, stream));
    }
    step += m;
  }
  HD_TRY(launch_swarm_reduce<P>(w, stream));
  double sums[2 * kNoAllocFields];
  uint64_t coll[kNoAllocFields], over[kNoAllocFields];
  HD_TRY(hipMemcpyAsync(sums, w.sums, 2 * D * 8, hipMemcpyDeviceToHost, stream));
  HD_TRY(hipMemcpyAsync(coll, w.coll, D * 8, hipMemcpyDeviceToHost, stream));
  HD_TRY(hipMemcpyAsync(over, w.over, D * 8, hipMemcpyDeviceToHost, stream));
  HD_TRY(hipStreamSynchronize(stream));
  swarm_fill_results(p, M, n_avg, sums, coll, over, out);
  return HD_OK;
}

}  // namespace

}  // namespace hd

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
struct hd_batch {
  hd::BatchBase* impl;
};
struct hd_discharge {
  hd_batch b;
};

namespace {

int make_batch(const hd_params* const* params, int32_t n, const hd_device_ctx* ctx,
               hd::BatchBase** out) {
  using namespace hd;
  if (!params || n < 1) return fail(HD_EINVAL, "no discharges");
  std::string why;
  for (int i = 0; i < n; ++i)
    if (!validate(params[i], why)) return fail(HD_EINVAL, "discharge " + std::to_string(i) + ": " + why);
  for (int i = 1; i < n; ++i)
    if (params[i]->precision != params[0]->precision ||
        params[i]->sort_every != params[0]->sort_every ||
        params[i]->eedf_every != params[0]->eedf_every)
      return fail(HD_EINVAL, "batch members must share precision, sort_every and eedf_every");
  BatchBase* b = nullptr;
  int rc;
  if (params[0]->precision == HD_FP32) {
    auto* x = new Batch<float>();
    x->precision = HD_FP32;
    rc = x->create(params, n, ctx);
    b = x;
  } else {
    auto* x = new Batch<double>();
    x->precision = HD_FP64;
    rc = x->create(params, n, ctx);
    b = x;
  }
  if (rc != HD_OK) {
    delete b;
    return rc;
  }
  *out = b;
  return HD_OK;
}

template <class F>
int dispatch(hd::BatchBase* b, F&& f) {
  if (b->precision == HD_FP32) return f(static_cast<hd::Batch<float>*>(b));
  return f(static_cast<hd::Batch<double>*>(b));
}

}  // namespace

extern "C" {

int32_t hd_abi_version(void) { return HD_ABI_VERSION; }
const char* hd_last_error(void) { return hd::g_err.c_str(); }

size_t hd_required_bytes(const hd_params* p) {
  std::string why;
  if (!hd::validate(p, why)) return 0;
  return p->precision == HD_FP32 ? hd::required_bytes<float>(*p) : hd::required_bytes<double>(*p);
}

int hd_init_discharge(const hd_params* params, const hd_device_ctx* ctx, hd_discharge** out) {
  if (!out) return hd::fail(HD_EINVAL, "null out");
  hd::BatchBase* b = nullptr;
  const hd_params* arr[1] = {params};
  int rc = make_batch(arr, 1, ctx, &b);
  if (rc) return rc;
  *out = new hd_discharge{hd_batch{b}};
  return HD_OK;
}

int hd_step(hd_discharge* h, int64_t n) {
  if (!h) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(h->b.impl, [&](auto* x) { return x->step(n); });
}

int hd_moments(hd_discharge* h, hd_moment_set* out) {
  if (!h) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(h->b.impl, [&](auto* x) { return x->moments(0, out); });
}

int hd_get_particles(hd_discharge* h, int32_t* cell, void* off, void* vx, void* vy, void* vz,
                     uint32_t* id, int64_t cap, int64_t* n_out) {
  if (!h) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(h->b.impl,
                  [&](auto* x) { return x->particles(0, cell, off, vx, vy, vz, id, cap, n_out); });
}

int hd_get_push_field(hd_discharge* h, void* ep) {
  if (!h || !ep) return hd::fail(HD_EINVAL, "null argument");
  return dispatch(h->b.impl, [&](auto* x) { return x->push_field(0, ep); });
}

struct hd_server {
  hd::ServerBase* impl;
};

int hd_server_create(const hd_server_config* cfg, const hd_device_ctx* ctx, hd_server** out) {
  if (!cfg || !out) return hd::fail(HD_EINVAL, "null argument");
  if ((cfg->precision != HD_FP32 && cfg->precision != HD_FP64) || cfg->max_slots < 1 ||
      cfg->max_slots > 1024 || cfg->sort_every < 1 || cfg->eedf_every < 1 ||
      cfg->max_cells < 2 || cfg->max_cells > hd::kMaxCells || cfg->max_energy < 2 ||
      cfg->max_channels < 0 || cfg->max_channels > HD_MAX_CHANNELS || cfg->max_eedf_bins < 1 ||
      cfg->hbm_budget_bytes == 0)
    return hd::fail(HD_EINVAL, "invalid server configuration");
  hd::ServerBase* s = nullptr;
  int rc;
  if (cfg->precision == HD_FP32) {
    auto* x = new hd::Server<float>();
    rc = x->create(cfg, ctx);
    s = x;
  } else {
    auto* x = new hd::Server<double>();
    rc = x->create(cfg, ctx);
    s = x;
  }
  if (rc) {
    delete s;
    return rc;
  }
  *out = new hd_server{s};
  return HD_OK;
}

int hd_server_submit(hd_server* s, const hd_params* p, int64_t n, uint64_t* job_id) {
  if (!s || !job_id) return hd::fail(HD_EINVAL, "null argument");
  return s->impl->submit(p, n, job_id);
}

int hd_server_poll(hd_server* s, uint64_t job_id, int32_t* state, hd_moment_set* out,
                   double* times) {
  if (!s) return hd::fail(HD_EINVAL, "null handle");
  return s->impl->poll(job_id, state, out, times);
}

int hd_server_stats(hd_server* s, hd_server_counters* out) {
  if (!s || !out) return hd::fail(HD_EINVAL, "null argument");
  return s->impl->stats(out);
}

int hd_server_drain(hd_server* s, double timeout_s) {
  if (!s) return hd::fail(HD_EINVAL, "null handle");
  return s->impl->drain(timeout_s);
}

int hd_server_cancel(hd_server* s, uint64_t job_id) {
  if (!s) return hd::fail(HD_EINVAL, "null server");
  return s->impl->cancel(job_id);
}

int hd_server_free(hd_server* s) {
  if (!s) return HD_OK;
  delete s->impl;
  delete s;
  return HD_OK;
}

int hd_profile_steps(hd_discharge* h, int64_t n, double* out_ms) {
  if (!h) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(h->b.impl, [&](auto* x) { return x->profile(n, out_ms); });
}

int hd_batch_profile_steps(hd_batch* b, int64_t n, double* out_ms) {
  if (!b) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(b->impl, [&](auto* x) { return x->profile(n, out_ms); });
}

int hd_grow(hd_discharge* h, int64_t new_capacity) {
  if (!h) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(h->b.impl, [&](auto* x) { return x->grow(new_capacity); });
}

int hd_save(hd_discharge* h, void* out, size_t capacity_bytes, size_t* used_bytes) {
  if (!h) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(h->b.impl, [&](auto* x) { return x->save(out, capacity_bytes, used_bytes); });
}

int hd_restore(hd_discharge* h, const void* in, size_t bytes) {
  if (!h) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(h->b.impl, [&](auto* x) { return x->restore(in, bytes); });
}

int hd_free(hd_discharge* h) {
  if (!h) return HD_OK;
  delete h->b.impl;
  delete h;
  return HD_OK;
}

int hd_batch_create(const hd_params* const* params, int32_t n, const hd_device_ctx* ctx,
                    hd_batch** out) {
  if (!out) return hd::fail(HD_EINVAL, "null out");
  hd::BatchBase* b = nullptr;
  int rc = make_batch(params, n, ctx, &b);
  if (rc) return rc;
  *out = new hd_batch{b};
  return HD_OK;
}

int hd_batch_step(hd_batch* b, int64_t n) {
  if (!b) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(b->impl, [&](auto* x) { return x->step(n); });
}

int hd_batch_moments(hd_batch* b, int32_t i, hd_moment_set* out) {
  if (!b) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(b->impl, [&](auto* x) { return x->moments(i, out); });
}

int hd_batch_get_particles(hd_batch* b, int32_t i, int32_t* cell, void* off, void* vx, void* vy,
                           void* vz, uint32_t* id, int64_t cap, int64_t* n_out) {
  if (!b) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(b->impl,
                  [&](auto* x) { return x->particles(i, cell, off, vx, vy, vz, id, cap, n_out); });
}

int hd_batch_free(hd_batch* b) {
  if (!b) return HD_OK;
  delete b->impl;
  delete b;
  return HD_OK;
}

int hd_batch_get_launch(hd_batch* b, hd_launch_config* out) {
  if (!b || !out) return hd::fail(HD_EINVAL, "null handle or output");
  *out = b->impl->launch;
  return HD_OK;
}

int hd_batch_set_launch(hd_batch* b, const hd_launch_config* cfg) {
  if (!b || !cfg) return hd::fail(HD_EINVAL, "null handle or configuration");
  if (b->impl->error) return hd::fail(b->impl->error, "handle is in an error state");
  return dispatch(b->impl, [&](auto* x) { return x->apply_launch(*cfg); });
}

int hd_batch_autotune(hd_batch* b, int64_t max_steps, hd_launch_config* out) {
  if (!b) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(b->impl, [&](auto* x) { return x->autotune(max_steps, out); });
}

int hd_get_launch(hd_discharge* h, hd_launch_config* out) {
  if (!h || !out) return hd::fail(HD_EINVAL, "null handle or output");
  *out = h->b.impl->launch;
  return HD_OK;
}

int hd_set_launch(hd_discharge* h, const hd_launch_config* cfg) {
  if (!h || !cfg) return hd::fail(HD_EINVAL, "null handle or configuration");
  if (h->b.impl->error) return hd::fail(h->b.impl->error, "handle is in an error state");
  return dispatch(h->b.impl, [&](auto* x) { return x->apply_launch(*cfg); });
}

int hd_autotune(hd_discharge* h, int64_t max_steps, hd_launch_config* out) {
  if (!h) return hd::fail(HD_EINVAL, "null handle");
  return dispatch(h->b.impl, [&](auto* x) { return x->autotune(max_steps, out); });
}

int hd_diag_arith(int32_t precision, int64_t n, const void* a, const void* b, void* out,
                  const hd_device_ctx* ctx) {
  if (n < 0 || (n > 0 && (!a || !b || !out))) return hd::fail(HD_EINVAL, "bad arguments");
  if (precision != HD_FP32 && precision != HD_FP64) return hd::fail(HD_EINVAL, "precision");
  if (n == 0) return HD_OK;
  hipStream_t s = ctx ? (hipStream_t)ctx->stream : nullptr;
  const size_t es = precision == HD_FP32 ? 4 : 8;
  void *da = nullptr, *db = nullptr, *dout = nullptr;
  auto cleanup = [&]() {
    if (da) (void)hipFree(da);
    if (db) (void)hipFree(db);
    if (dout) (void)hipFree(dout);
  };
  if (hipMalloc(&da, n * es) != hipSuccess || hipMalloc(&db, n * es) != hipSuccess ||
      hipMalloc(&dout, 4 * n * es) != hipSuccess) {
    cleanup();
    return hd::fail(HD_ENOMEM, "diag allocation failed");
  }
  hipError_t e = hipMemcpy(da, a, n * es, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(db, b, n * es, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = precision == HD_FP32
            ? hd::launch_diag<float>(n, (const float*)da, (const float*)db, (float*)dout, s)
            : hd::launch_diag<double>(n, (const double*)da, (const double*)db, (double*)dout, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(out, dout, 4 * n * es, hipMemcpyDeviceToHost);
  cleanup();
  if (e != hipSuccess) return hd::fail(HD_EDEVICE, hipGetErrorString(e));
  return HD_OK;
}

struct hd_swarm {
  hd::SwarmBase* impl;
};

int hd_swarm_run_noalloc(const hd_swarm_params* params, int64_t n_relax, int64_t n_avg,
                         const hd_device_ctx* ctx, hd_swarm_result* out) {
  if (!out) return hd::fail(HD_EINVAL, "null output");
  if (n_relax < 0 || n_avg < 0) return hd::fail(HD_EINVAL, "step counts must be non-negative");
  std::string why;
  if (!hd::swarm_valid(params, why)) return hd::fail(HD_EINVAL, why);
  if (ctx && ctx->arena) return hd::fail(HD_EINVAL, "the ion swarm takes no arena");
  const int device = ctx ? ctx->device : 0;
  hipStream_t stream = ctx ? (hipStream_t)ctx->stream : nullptr;
  if (hipSetDevice(device) != hipSuccess) return hd::fail(HD_EDEVICE, "hipSetDevice");
  return params->precision == HD_FP32
             ? hd::swarm_noalloc<float>(*params, n_relax, n_avg, stream, device, out)
             : hd::swarm_noalloc<double>(*params, n_relax, n_avg, stream, device, out);
}

int hd_swarm_create(const hd_swarm_params* params, const hd_device_ctx* ctx, hd_swarm** out) {
  if (!out) return hd::fail(HD_EINVAL, "null out");
  std::string why;
  if (!hd::swarm_valid(params, why)) return hd::fail(HD_EINVAL, why);
  if (ctx && ctx->arena) return hd::fail(HD_EINVAL, "the ion swarm takes no arena");
  hd::SwarmBase* b = nullptr;
  int rc;
  if (params->precision == HD_FP32) {
    auto* x = new hd::SwarmImpl<float>();
    rc = x->create(params, ctx);
    b = x;
  } else {
    auto* x = new hd::SwarmImpl<double>();
    rc = x->create(params, ctx);
    b = x;
  }
  if (rc) {
    delete b;
    return rc;
  }
  *out = new hd_swarm{b};
  return HD_OK;
}

int hd_swarm_run(hd_swarm* h, int64_t n_steps, int32_t accumulate) {
  if (!h) return hd::fail(HD_EINVAL, "null handle");
  return h->impl->run(n_steps, accumulate);
}

int hd_swarm_results(hd_swarm* h, hd_swarm_result* out) {
  if (!h) return hd::fail(HD_EINVAL, "null handle");
  return h->impl->results(out);
}

int hd_swarm_get_ions(hd_swarm* h, int32_t field, void* vx, void* vy, void* vz, double* acc_vz,
                      double* acc_v2, int64_t cap) {
  if (!h) return hd::fail(HD_EINVAL, "null handle");
  return h->impl->ions(field, vx, vy, vz, acc_vz, acc_v2, cap);
}

int hd_swarm_free(hd_swarm* h) {
  if (!h) return HD_OK;
  delete h->impl;
  delete h;
  return HD_OK;
}

}  // extern "C"
