// Internal layout of the discharge state in device memory, shared by the
// kernels and the host runtime of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hd {

constexpr int kMaxK = 16;          // collision channels
constexpr int kThreads = 256;      // append workgroup
constexpr int kPerThread = 4;      // particles per thread per chunk (vector loads)
constexpr int kElecThreads = 512;  // electron-kernel workgroup (8 waves)
constexpr int kTile = kElecThreads * kPerThread;  // particles per chunk
constexpr int kSub = 64 * kPerThread;  // particles of one wave in a chunk (a sub-chunk)
constexpr int kElecWide = 8;  // electron launch variants kElecWide + v: kernel v, 1,024-thread workgroups
constexpr int kSeeMax = 4096;      // secondaries per wall per step
constexpr int kMaxCells = 4096;    // cells per discharge
constexpr int kMaxNodes = kMaxCells + 1;
constexpr int kMaxSegs = 4096;    // particle workgroups of one electron launch
constexpr int kSphereTries = 64;   // bound of the rejection loops
constexpr int kSortTile = 4096;    // items per sort tile (one workgroup of the sort)
constexpr int kFinThreads = 1024;  // field/finalize workgroup
constexpr int kMaxSpecies = 4;     // ion species of the multi-species model
constexpr int kMaxMu = 256;        // mobility-table points per species

// Mutable per-discharge scalars.  They live in device memory so that a
// captured sequence of launches can advance without host involvement.
struct State {
  int64_t step;          // completed steps
  int64_t steps_left;    // steps still to run in the current request (<= 0: idle)
  uint32_t n_main;       // particle slots in use (holes included)
  uint32_t next_id;      // id of the next appended particle
  uint32_t append_base;  // first slot of this step's appended particles
  uint32_t id_base;      // id of this step's first appended particle
  uint32_t n_kids;       // children created this step
  uint32_t n_see[2];     // secondaries emitted this step (left, right)
  uint32_t n_chunks;     // sub-chunks processed by the last electron launch
  uint32_t seg_off;      // launch-wide index of this discharge's first chunk (last launch)
  uint32_t seg_per;      // chunks per particle workgroup (last launch)
  int32_t fin_ready;     // set by the end-of-step workgroup once its offsets are published
  uint32_t app_done;     // append workgroups finished with this discharge (this launch)
  int32_t buf;           // current particle buffer (0/1)
  int32_t cbuf;          // cnt buffer holding the deposit of the current step
  int32_t error;         // sticky error (HD_E* code)
  int32_t sort_due;      // set by the finalize kernel when a sort follows
  int32_t append_pending;  // set by the finalize kernel when particles are to be appended
  uint32_t n_live_sorted;  // live particles counted by the sort
  double wall[2];        // ion wall fluxes Gamma_0, Gamma_N of the last fluid update
                         // (several species: the net charge flux sum_s Z_s Gamma_s)
  double see_flux[2];    // several species: positive-ion flux into each wall
  uint64_t coll[kMaxK];
  uint64_t absorbed[2];
  uint64_t emitted[2];
  uint64_t created;
  uint64_t overflow;
  uint64_t see_clamped;
  uint64_t n_acc;
  uint64_t pushed;  // live particles pushed (particle-steps) since creation
  // RF drive and absorbed power (Eq 2.9)
  double volt_amp;     // amplitude of the current RF period [V]
  double pw_sum;       // sum over the current period's steps of V J [W/m^2]
  double p_abs;        // period-averaged absorbed power of the last period [W/m^2]
  int64_t rf_periods;  // completed RF periods
  uint64_t pw_abs0;    // electrons absorbed at z = 0 up to the end of the last step
  uint64_t pw_emi0;    // secondaries emitted at z = 0 up to the end of the last step
  // capacity checkpoints (rolling back an overflowing step)
  int64_t error_step;  // the step in which the error arose
  int64_t ckpt_step;   // the step at which the valid checkpoint was taken
  int32_t ckpt_due;    // checkpoint the coming interval's start (close to capacity)
  int32_t ckpt_valid;  // the checkpoint area holds the start of the current interval
  uint32_t prev_n_main;  // slots in use at the last interval's start
  uint32_t pad1;
};

// Immutable constants and device pointers of one discharge.
template <class P>
struct Disch {
  int32_t nc, nn, ne, K;
  int32_t nbins, sort_every, eedf_every, ion_model;
  uint32_t capacity;        // slots per particle buffer (multiple of kTile)
  uint32_t cap_sub;         // capacity / kSub
  uint32_t sort_tiles_max;  // capacity / kSortTile (rounded up)
  uint32_t pad0;
  uint64_t seed;
  // electron constants rounded to P
  P Pmax, KE, invKE, inv_dE, kdz, delta, keedf;
  P thr[kMaxK];
  P delta_k[kMaxK];      // elastic recoil 2 m_e / M_target per channel
  int32_t kind[kMaxK];
  int32_t product[kMaxK];  // ion species of an ionization / attachment
  uint32_t ion_mask;       // bit k: channel k is an ionization
  uint32_t att_mask;       // bit k: channel k is an attachment
  // FP64 constants of the field, fluid and emission
  double dz, L, w, kp, inv_dz, inv_2dz, hdz_eps, qm_dt, scale_in, scale_wall;
  double mu, nu, mu_full, TN, kappa, M, dt, dt_2dz, dt_dz, e_M_dt, dt_2dzM, hdt, nfloor;
  double gamma_see, see_v;  // emission coefficient and speed sqrt(E_sec 2e/m_e)
  double power_P0, power_alpha;  // Eq 2.9 (power_P0 = 0: fixed amplitude)
  // ion species (S = 1 for the single-species models: Z = +1)
  int32_t S;
  int32_t Z[kMaxSpecies];
  int32_t n_mu[kMaxSpecies];
  double kappa_s[kMaxSpecies];                // Eq (2.8) factor per species
  double mu_lo[kMaxSpecies], mu_L0[kMaxSpecies], mu_inv_dL[kMaxSpecies];
  const double* mu_tab;                       // [S * kMaxMu] mobility tables
  double n_gas;
  int64_t rf_steps;              // steps per RF period (0: no period ends)
  int64_t volt_len;
  // tables
  const double* ip;    // [nn] inverse Thomas pivots of the Poisson matrix
  const P* tab;        // [ne*K] cumulative collision probabilities
  const double* volt;  // [volt_len] unit drive waveform sin(2 pi f t_n + phase) per step
  // particles: two buffers for out-of-place sorting
  int32_t* cell[2];
  P* off[2];
  P* vx[2];
  P* vy[2];
  P* vz[2];
  uint32_t* id[2];
  // children staging: sub-chunk k writes its children at [k*kSub, ...)
  int32_t* kc;
  P* koff;
  P* kvx;
  P* kvy;
  P* kvz;
  uint32_t* chunk_kids;  // [cap_sub] children per sub-chunk
  uint32_t* chunk_base;  // [cap_sub] their offset among the children of the sub-chunk's workgroup
  uint32_t* seg;         // [kMaxSegs] children per particle workgroup, then their offsets
  // secondaries of this step: side s at [s*kSeeMax, ...)
  int32_t* sc;
  P* soff;
  P* svx;
  P* svy;
  P* svz;
  // grids
  int64_t* cnt[2];
  int64_t* ion_src;  // [S * nn]
  double* ni;        // [S * nn]
  double* gam;       // [S * nn]
  double* phi;
  double* E;
  P* Ep;
  double* scratch;  // [12*nn] solver work space
  uint64_t* acc_cnt;
  double* acc_ni;
  uint64_t* eedf;  // [nbins+1]
  // sort
  uint32_t* hist;  // [nc * sort_tiles_max]
  uint32_t* bin_start;  // scan partials
  int32_t* tile_rng;    // [2 * sort_tiles_max] lowest / highest live cell of each tile
  State* st;
  // checkpoint area: a copy of the grid region (grid_bytes from cnt[0] on:
  // deposits, ion sources, densities, fluxes, fields, run sums, EEDF) and,
  // at ckpt + grid_bytes, of the State
  unsigned char* ckpt;
  uint64_t grid_bytes;
};

// Auxiliary ion swarm: n_fields independent swarms of n_ions ions, ion i of
// swarm f at index f * n_ions + i of every array.
constexpr int kSwarmThreads = 256;
constexpr int kSwarmMaxEnergy = 4096;  // rate-table points held in LDS (32 KB in FP64)
template <class P>
struct SwarmDev {
  int32_t n_fields, ne;
  int64_t n_ions;
  uint64_t seed;
  P Pmax, KEr, inv_dE, m1, m2;  // null-collision bound, M_r/(2e), points per eV, mass ratios
  double vth_n, vth_i0;         // thermal speeds of gas atoms and of the initial ions
  const P* a;                   // [n_fields] velocity gain per step e E0 dt / M
  const P* tab;                 // [ne] P_max nu(eps_i) / nu_max
  P* vx;
  P* vy;
  P* vz;
  double* avz;    // per-ion sums of v_z over accumulated steps
  double* av2;    // per-ion sums of |v|^2
  uint64_t* coll;  // [n_fields]
  uint64_t* over;  // [n_fields]
  double* sums;    // [2 n_fields] sums over ions of avz and av2
};

}  // namespace hd

// Launch wrappers implemented in the kernel translation units.
namespace hd {
template <class P>
hipError_t launch_finalize(const Disch<P>* d_dev, int D, int field_only, int nn_max,
                           int app_blocks, hipStream_t s);
template <class P>
hipError_t launch_diag(int64_t n, const P* a, const P* b, P* out, hipStream_t s);
template <class P>
hipError_t launch_swarm_init(const SwarmDev<P>& w, hipStream_t s);
template <class P>
hipError_t launch_swarm_step(const SwarmDev<P>& w, uint32_t step0, int n_steps, int accumulate,
                             hipStream_t s);
template <class P>
hipError_t launch_swarm_reduce(const SwarmDev<P>& w, hipStream_t s);
template <class P>
hipError_t launch_swarm_clear(const SwarmDev<P>& w, hipStream_t s);
}  // namespace hd
