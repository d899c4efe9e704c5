/*
 * hd.h -- C ABI of the MI355X (gfx950) hybrid PIC/MCC discharge stepper.
 *
 * Method: Eremin, Hemke & Mussenbrock, "A New Hybrid Scheme for Simulations
 * of Highly Collisional RF-Driven Plasmas" (arXiv 1508.02892).  A 1D
 * parallel-plate discharge (powered electrode at z = 0, grounded at z = L,
 * Sec. II) with kinetic 1D3V PIC/MCC electrons (Sec. II.A) and a fluid ion
 * species (Sec. II.B full model, Eqs 2.3-2.4; Sec. II.C drift-diffusion,
 * Eqs 2.4-2.8), coupled through Poisson's equation, impact ionization and
 * ion-induced secondary emission (Sec. II.D).
 *
 * Every step of the time loop runs in HIP kernels on the device; the host
 * only validates parameters, computes derived constants and collision
 * tables, performs the initial particle load and enqueues work.
 *
 * Conventions
 *  - All functions return HD_OK (0) or a negative HD_E* code and never throw.
 *    hd_last_error() returns a thread-local description of the last failure.
 *  - Handles are not thread-safe: one handle is driven by one host thread,
 *    and its work is enqueued on the stream given at creation.
 *  - "Caller-owned" buffers are host memory unless stated otherwise; the
 *    library copies what it needs and never keeps caller pointers.
 *  - Units are SI except energies, which are in eV.
 */
#ifndef HD_H
#define HD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HD_ABI_VERSION 4

enum hd_status {
  HD_OK = 0,
  HD_EINVAL = -1,     /* invalid or inconsistent parameters / arguments      */
  HD_ENOMEM = -2,     /* device allocation failed or arena too small          */
  HD_EDEVICE = -3,    /* HIP runtime error (sticky for the handle)            */
  HD_ECAPACITY = -4,  /* particle capacity exceeded.  One discharge: the handle
                         is rolled back to the last complete step and
                         hd_grow then continues the run (see hd_step).
                         Batches and served jobs: the discharge stops.      */
  HD_ENUMERIC = -5,   /* the field of the next step is not finite (checked at
                         every node at the end of every step); the handle
                         refuses further steps                               */
  HD_ESTATE = -6,     /* operation not valid in the handle's current state    */
  HD_ESYNC = -7       /* a bounded wait of one workgroup for another of the
                         same launch ran out (the device did not keep the
                         end-of-step workgroup resident beside the append
                         workgroups); the handle refuses further steps      */
};

enum hd_precision { HD_FP32 = 0, HD_FP64 = 1 };

/* Ion model: drift-diffusion (Sec. II.C, explicit option) or the full fluid
 * with inertia (Sec. II.B, Eq 2.3 solved by a tridiagonal solve), each with a
 * constant transport coefficient (mu_const / nu_const) or with the fitted
 * He+-in-He coefficients at atmospheric pressure: the mobility as a function
 * of the local |E| (Table 2) for drift-diffusion, the momentum-exchange
 * frequency as a function of the lagged local |u| (Table 3) for the full
 * fluid, with mu = e/(M nu) in the wall fluxes and Eq (2.8).  The fitted
 * models ignore mu_const / nu_const. */
enum hd_ion_model {
  HD_ION_DD_CONST_MU = 0,
  HD_ION_FULL_CONST_NU = 1,
  HD_ION_DD_FIT_MU = 2,
  HD_ION_FULL_FIT_NU = 3,
  HD_ION_DD_SPECIES = 4   /* several drift-diffusion species, see hd_ion_species */
};

/* Electron-neutral reaction kinds (Table 1: R1 elastic, R2 ionization,
 * R3 excitation), and attachment: the electron is lost to a negative ion
 * (the removal of Sec. II.D applied to attachment). */
enum hd_xs_kind {
  HD_XS_ELASTIC = 0,
  HD_XS_EXCITATION = 1,
  HD_XS_IONIZATION = 2,
  HD_XS_ATTACHMENT = 3
};

#define HD_MAX_CHANNELS 16
#define HD_MAX_SPECIES 4

/* One electron-neutral channel.  sigma_m2 holds n_energy cross sections [m^2]
 * on the uniform grid E_i = i / inv_de_per_eV (caller-owned, copied).  The
 * channel's collision frequency is (n_gas_m3 target_fraction) sigma v. */
typedef struct hd_xs_channel {
  int32_t kind;          /* enum hd_xs_kind                                  */
  int32_t product;       /* ion species that receives the ion of an
                            ionization (charge +1) or attachment (charge -1);
                            0 for the single-species ion models            */
  double threshold_eV;   /* energy lost in excitation / ionization           */
  const double* sigma_m2;
  double target_fraction; /* share of n_gas_m3 that is this channel's target,
                             in [0, inf) (1: the whole gas)                  */
  double target_mass_amu; /* target mass of the elastic recoil 2 m_e / M
                             (0: m_gas_amu)                                 */
} hd_xs_channel;

/* One ion species of HD_ION_DD_SPECIES: drift-diffusion (Sec. II.C, Eq 2.5
 * with the charge sign) with a mobility tabulated against E/N on n_mu
 * log-spaced points from en_lo_Td to en_hi_Td (1 Td = 1e-21 V m^2),
 * interpolated linearly in ln(E/N) and held at the end values outside;
 * Eq (2.8) with the species' mass; the wall flux is kept only when the
 * drift points into the wall.  The species starts at init_fraction times
 * the initial electron density. */
typedef struct hd_ion_species {
  int32_t charge;        /* +1 or -1                                         */
  int32_t n_mu;          /* 2 .. 256                                         */
  double m_amu;
  double en_lo_Td, en_hi_Td;
  const double* mu_m2_Vs; /* [n_mu] (caller-owned, copied)                   */
  double init_fraction;
} hd_ion_species;

/* Problem statement of one discharge (caller-owned, copied at creation). */
typedef struct hd_params {
  int32_t abi_version;   /* must be HD_ABI_VERSION                           */
  int32_t precision;     /* enum hd_precision: particle state and MCC math   */
  int32_t ion_model;     /* enum hd_ion_model                                */
  int32_t n_cells;       /* N_c >= 2 uniform cells; nodes j = 0 .. N_c       */
  int32_t n_energy;      /* collision-table points (>= 2)                    */
  int32_t n_channels;    /* 0 .. HD_MAX_CHANNELS                             */
  int32_t sort_every;    /* compaction + stable cell sort every this many steps */
  int32_t eedf_every;    /* EEDF sample every this many steps                */
  int32_t n_eedf_bins;   /* EEDF bins over [0, eedf_emax_eV)                 */
  int32_t n_species;     /* HD_ION_DD_SPECIES: 1 .. HD_MAX_SPECIES; else 0   */
  int64_t n_macro;       /* N_0 initial electron superparticles              */
  int64_t capacity;      /* particle slots reserved (>= n_macro)             */
  uint64_t seed;         /* Philox key                                       */
  /* background gas: uniform, constant (Sec. II.A) */
  double n_gas_m3, t_gas_K, m_gas_amu;
  /* geometry */
  double gap_m;
  /* drive: V(t_n) = U sin(2 pi f_rf_Hz t_n + phase_rad) at z = 0, t_n = n dt_s,
     U = v_amp_V unless power control (below) adjusts it */
  double v_amp_V, f_rf_Hz, phase_rad;
  /* electron load: uniform in [load_lo L, load_hi L), Maxwellian t_e0_eV;
     superparticle weight from Eq 1.2 */
  double n_e0_m3, t_e0_eV, load_lo, load_hi;
  /* ion-induced secondary emission (Sec. II.D) */
  double gamma_see, e_sec_eV;
  /* ions: mass, constant mobility (DD) or momentum-exchange frequency (full) */
  double m_ion_amu, mu_const, nu_const;
  /* numerics */
  double dt_s;
  double inv_de_per_eV;  /* collision-table points per eV                    */
  double eedf_emax_eV;
  /* Power control (Sec. II.D, Eq 2.9).  An RF period is round(1/(f_rf_Hz
     dt_s)) steps.  Every step adds to the period's sum the power delivered
     at z = 0 over [t_n, t_n+1]: (V_n + V_n+1)/2 times the current density
     e (Gamma_i - Gamma_e) + eps0 (E_0^{n+1} - E_0^n)/dt_s, with Gamma_i the
     ion wall flux of the step and Gamma_e = w (emitted - absorbed electrons
     at z = 0 in the step)/dt_s; the interval counts for the period that
     holds t_n+1.  P_abs = sum / steps per period.  With power_W_m2 > 0 the
     amplitude of the next period is U (1 - power_alpha (P_abs - P_0)/P_0),
     P_0 = power_W_m2; with 0 the amplitude stays v_amp_V (P_abs is still
     reported).  power_W_m2 > 0 needs a period of at least 2 steps. */
  double power_W_m2;     /* P_0 / S, prescribed absorbed power [W/m^2], >= 0 */
  double power_alpha;    /* alpha of Eq 2.9, >= 0                            */
  const hd_xs_channel* channels; /* n_channels entries, caller-owned, copied */
  const hd_ion_species* species; /* n_species entries, caller-owned, copied  */
} hd_params;

/* Device context.  stream: a hipStream_t (NULL: the library creates a
 * non-blocking stream of its own).  device: HIP device ordinal.  arena:
 * device memory of the caller (on that device) from which a discharge or
 * batch takes all of its device state instead of calling hipMalloc, at
 * least the sum of hd_required_bytes of its discharges; runs past 32,768
 * steps also take 8 bytes per step of the drive table from it, in doubling
 * increments (HD_ENOMEM from hd_step when it is exhausted).  The caller
 * keeps the arena alive and unused until the handle is freed.  NULL: the
 * library allocates.  The server and the ion swarm take no arena
 * (HD_EINVAL). */
typedef struct hd_device_ctx {
  void* stream;
  int32_t device;
  int32_t reserved;
  void* arena;
  size_t arena_bytes;
} hd_device_ctx;

/* Moments of one discharge (Sec. III reports density profiles and the EEDF).
 * Array pointers are caller-owned host buffers sized as noted; any may be
 * NULL to skip it.  hd_moments fills the scalar fields and the non-NULL
 * arrays. */
typedef struct hd_moment_set {
  int64_t step;            /* completed steps                                */
  int64_t n_live;          /* live electron superparticles                   */
  int64_t n_slots;         /* particle slots in use, including holes         */
  int32_t n_nodes;         /* N_c + 1                                        */
  int32_t n_channels;
  int32_t n_eedf_bins;
  int32_t error;           /* device-side sticky error (0 = none)            */
  double* n_e;             /* [n_nodes] electron density of the current step */
  double* n_i;             /* [n_nodes] ion charge density / e: n_i, or with
                              several species sum_s charge_s n_s           */
  double* phi;             /* [n_nodes] potential of the current step [V]    */
  double* E;               /* [n_nodes] field of the current step [V/m]      */
  double* gamma_i;         /* [n_nodes] last ion flux [m^-2 s^-1] (several
                              species: sum_s charge_s Gamma_s)              */
  double* n_e_avg;         /* [n_nodes] average of n_e over completed steps  */
  double* n_i_avg;         /* [n_nodes] average of n_i over completed steps  */
  double* n_species;       /* [n_species * n_nodes] species densities, or NULL */
  double* gamma_species;   /* [n_species * n_nodes] species fluxes, or NULL  */
  int64_t* cnt;            /* [n_nodes] fixed-point deposit (2^32 per particle) */
  uint64_t* eedf_counts;   /* [n_eedf_bins + 1], last entry = overflow       */
  double* eedf;            /* [n_eedf_bins] normalised: sum f dE = 1         */
  uint64_t coll[HD_MAX_CHANNELS];  /* collisions per channel                 */
  uint64_t absorbed[2];    /* electrons absorbed at z = 0 / z = L            */
  uint64_t emitted[2];     /* secondaries emitted at z = 0 / z = L           */
  uint64_t created;        /* electrons created by ionization                */
  uint64_t e_overflow;     /* collision candidates above the table's top     */
  uint64_t see_clamped;    /* secondaries dropped by the per-step cap        */
  uint64_t n_acc;          /* steps in the averages                          */
  uint64_t pushed;         /* particle-steps: live electrons pushed, summed
                              over all steps so far                          */
  double volt_amp;         /* drive amplitude U of the coming steps [V]      */
  double p_abs;            /* P_abs of the last completed RF period [W/m^2]  */
  int64_t rf_periods;      /* completed RF periods                           */
  int64_t graph_steps;     /* steps of this handle replayed from captured
                              launch graphs (the rest were launched one
                              kernel at a time)                              */
  int64_t rollbacks;       /* capacity overflows rolled back (hd_step)       */
} hd_moment_set;

typedef struct hd_batch hd_batch;
typedef struct hd_discharge hd_discharge;

/* ---- library ------------------------------------------------------------ */

int32_t hd_abi_version(void);
const char* hd_last_error(void);

/* Device bytes one discharge with these parameters occupies: its state
 * block (two particle buffers of `capacity` slots, staging, grids, tables,
 * the drive table of the first 32,768 steps) and its descriptor (Sec. II.A
 * particles and Secs. II.B-D grids); 0 if the parameters are invalid
 * (hd_last_error says why). */
size_t hd_required_bytes(const hd_params* params);

/* ---- one discharge (Sec. II) -------------------------------------------- */

/* Validates params, builds the null-collision tables (Sec. II.A), loads the
 * electrons (Eqs 1.1-1.2) and ions, allocates device state and computes the
 * field of step 0.  Synchronous.  *out is set only on HD_OK. */
int hd_init_discharge(const hd_params* params, const hd_device_ctx* ctx, hd_discharge** out);

/* Enqueues n_steps >= 0 time steps on the handle's stream and returns
 * without waiting.  Each step (Sec. II, the scheme's time step): the ion
 * fluid (Eqs 2.3-2.8) and the electron push / removal / null-collision
 * Monte Carlo / cloud-in-cell deposit (Sec. II.A), then emission and ion
 * sources (Sec. II.D), run averages, appending, the field of the next step
 * (Sec. II.D), and every sort_every steps a compaction and stable cell sort.
 * Errors of earlier steps surface here or at the next synchronising call.
 * Capacity: while a sort interval starts with the particle slots close to
 * `capacity`, the handle keeps a checkpoint of that interval's start; if
 * the interval then overflows, the next synchronising call restores the
 * checkpoint, replays the steps before the overflowing one (bitwise the
 * same run) and returns HD_ECAPACITY with the handle at the last complete
 * step (hd_moments then reports it); hd_grow raises the capacity and
 * hd_step continues.  Without a checkpoint the handle refuses further
 * steps. */
int hd_step(hd_discharge* h, int64_t n_steps);

/* Raises the particle capacity of a discharge to new_capacity (>= the
 * current one): reallocates its state block and copies the state
 * (synchronous).  Clears a rolled-back HD_ECAPACITY.  With an arena, the
 * new block is taken from the arena's unused part. */
int hd_grow(hd_discharge* h, int64_t new_capacity);

/* Snapshot and resume of a run (the state of Sec. II at a step boundary:
 * particles, ion fluid, fields, run sums).  hd_save waits for the handle's
 * stream and writes the discharge's state -- the state record, the particle
 * slots in use and the grids -- into the caller's host buffer out of
 * capacity_bytes; *used_bytes gets the snapshot's size (out = NULL only
 * queries it).  hd_restore loads a snapshot into a handle created with the
 * same parameters (capacity may differ; HD_ECAPACITY if the snapshot's slots
 * do not fit, hd_grow first), which then stands at the snapshot's step.  The
 * random streams are keyed by particle id and step (Sec. II.A), so a
 * resumed run is bitwise the uninterrupted one.  HD_EINVAL for a buffer
 * that is too small, not a snapshot of this library and precision, or of a
 * discharge with other parameters; a handle in an error state refuses
 * both.  Single discharges only. */
int hd_save(hd_discharge* h, void* out, size_t capacity_bytes, size_t* used_bytes);
int hd_restore(hd_discharge* h, const void* in, size_t bytes);

/* Waits for the handle's stream and fills *out (see hd_moment_set). */
int hd_moments(hd_discharge* h, hd_moment_set* out);

/* Waits and copies the particle slots [0, n_slots) into caller-owned host
 * arrays of length cap: cell (int32; -1 marks a hole), off/vx/vy/vz (float
 * for HD_FP32, double for HD_FP64), id (uint32).  *n_out = n_slots.  Any
 * array may be NULL.  HD_EINVAL if cap < n_slots. */
int hd_get_particles(hd_discharge* h, int32_t* cell, void* off, void* vx, void* vy, void* vz,
                     uint32_t* id, int64_t cap, int64_t* n_out);

/* Waits and copies E' = (-e/m_e) dt E at the nodes, rounded to the particle
 * precision (float or double array of n_nodes), as used by the next push. */
int hd_get_push_field(hd_discharge* h, void* ep);

/* Releases the device state of a discharge created by hd_init_discharge
 * (the discharge of Sec. II) and waits for its stream.  NULL-safe. */
int hd_free(hd_discharge* h);

/* ---- many independent discharges in one launch per phase ---------------- */

/* All discharges of a batch share precision, sort_every and eedf_every;
 * gap, grid, particle count, drive and seed may differ.  Each discharge's
 * result is bitwise identical to a one-discharge run of the same params. */
int hd_batch_create(const hd_params* const* params, int32_t n, const hd_device_ctx* ctx,
                    hd_batch** out);
int hd_batch_step(hd_batch* b, int64_t n_steps);
int hd_batch_moments(hd_batch* b, int32_t index, hd_moment_set* out);
int hd_batch_get_particles(hd_batch* b, int32_t index, int32_t* cell, void* off, void* vx,
                           void* vy, void* vz, uint32_t* id, int64_t cap, int64_t* n_out);
int hd_batch_free(hd_batch* b);

/* ---- launch shapes and the autotuner ------------------------------------- */

/* How the kernels of one handle are launched.  No field changes any result:
 * particles are processed in fixed sub-chunks of 256 (one wave's four
 * particles per lane), and every order that reaches a result (deposit sums
 * in 64-bit integers, children in parent order, a stable sort) is
 * independent of the launch shape, so results are bitwise identical
 * under every valid configuration.  A value of 0 selects the default; a new
 * handle starts from the autotuner's cached choice for its shape if there
 * is one, else from the defaults with electron variant 5 when its initial
 * particle state exceeds the 256 MB MALL and 0 otherwise, each moved to its
 * wide form (variant + 8) when the grid is so large that the LDS of a
 * 512-thread workgroup leaves room for only one per compute unit. */
typedef struct hd_launch_config {
  int32_t electron_variant; /* 0: each chunk of particles is loaded after the
                               previous chunk's stores have drained (FP32:
                               four waves per SIMD); 1: the next chunk's
                               loads stay in flight while a chunk is worked
                               on (FP32: three waves per SIMD); 2: loads
                               issued without the drain; 3, 4: as 0 and 2
                               with the nontemporal hint on the particle
                               loads and write-backs, which pays when the
                               particle store is far larger than the 256 MB
                               MALL and costs when it would stay there;
                               5, 6: as 3 and 4 with the hint on ids, cells
                               and offsets only (the velocities, which the
                               collision handler rewrites, stay cached);
                               7: as 3, with each chunk's collisions handled
                               before its velocities are written, in whole
                               64-byte segments.  These use 512-thread
                               workgroups (chunks of 2,048 particles);
                               8 + v: variant v with 1,024-thread workgroups
                               (chunks of 4,096), one per compute unit with
                               four waves per SIMD where large grids leave
                               LDS for only one narrow workgroup (the
                               autotuner also tries them when the particle
                               state exceeds the MALL); FP32 only, and not
                               for variant 1 (9 is rejected)               */
  int32_t electron_groups;  /* particle workgroups of the electron launch,
                               1 .. 4096 (0: as many as fit on the device at
                               once)                                       */
  int32_t sort_groups;      /* workgroups of the sort's launches, 1 .. 65536
                               (0: four per compute unit)                  */
  int32_t append_groups;    /* workgroups that append new particles in the
                               end-of-step launch, 1 .. compute units
                               (0: a quarter of the compute units)         */
  int32_t sort_tile;        /* particle slots per tile of the sort (one
                               workgroup's share): 4096 or 8192
                               (0: 4096)                                   */
} hd_launch_config;

/* Current configuration with defaults resolved to actual counts. */
int hd_batch_get_launch(hd_batch* b, hd_launch_config* out);
/* Validates and applies cfg to the following steps (HD_EINVAL if out of
 * range or if a variant cannot be resident with this batch's LDS needs). */
int hd_batch_set_launch(hd_batch* b, const hd_launch_config* cfg);
/* Autotuner.  Advances the batch by up to max_steps real steps (whole sort
 * intervals, at least two), launched one kernel at a time and timed with
 * HIP events on the handle's stream: each electron candidate (variant and
 * workgroup count) runs a block of consecutive steps whose first step is
 * not timed (a variant leaves the caches in its own state), the sort's
 * shapes (workgroup count and tile: 4096 or 8192) and the append's
 * workgroup counts are taken in turn, and each is given the fastest mean.  The
 * steps are ordinary steps of the run (the shapes do not change results).
 * The choice is applied, written to *out (may be NULL) and kept in a
 * process-wide cache keyed by the device and the batch's shape (precision,
 * discharges, particle count to a power of two, largest grid, channels,
 * ion models), which later handles with the same key start from.  If the
 * environment names a file in HD_TUNE_CACHE, the cache is also read from
 * and appended to that file. */
int hd_batch_autotune(hd_batch* b, int64_t max_steps, hd_launch_config* out);

/* The same for one discharge. */
int hd_get_launch(hd_discharge* h, hd_launch_config* out);
int hd_set_launch(hd_discharge* h, const hd_launch_config* cfg);
int hd_autotune(hd_discharge* h, int64_t max_steps, hd_launch_config* out);

/* ---- served job stream (continuous batching) ----------------------------- */

/* A server owns max_slots discharge slots on one device.  A host thread admits
 * submitted jobs first-come first-served into free slots while the device
 * bytes of the admitted jobs stay within hbm_budget_bytes, advances all
 * occupied slots together one sort interval (sort_every steps) per launch
 * sequence, and retires a job once it has run its steps, keeping its final
 * moments.  Jobs start at interval boundaries, so each job's result is
 * bitwise identical to the same discharge run alone.  Every job must match
 * the server's precision, sort_every and eedf_every and fit its caps.  An
 * interval runs with electron variant 5 (nontemporal traffic of ids, cells
 * and offsets) when the admitted jobs' initial particle state exceeds the
 * 256 MB MALL, else with variant 0, each in its wide form (13, 8) when the
 * slots' largest grid leaves LDS for only one 512-thread workgroup per
 * compute unit. */
typedef struct hd_server hd_server;

typedef struct hd_server_config {
  int32_t precision;        /* enum hd_precision of every job              */
  int32_t max_slots;        /* discharges resident at once (>= 1)          */
  int32_t sort_every;       /* steps per interval                          */
  int32_t eedf_every;
  int32_t max_cells;        /* caps that size the kernels' LDS             */
  int32_t max_energy;
  int32_t max_channels;
  int32_t max_eedf_bins;
  int32_t allow_full_fluid; /* admit HD_ION_FULL_CONST_NU jobs             */
  int32_t reserved;
  uint64_t hbm_budget_bytes;/* bound on the summed device bytes of the jobs */
} hd_server_config;

typedef struct hd_server_counters {
  uint64_t submitted, completed, failed, queued, running;
  uint64_t intervals;       /* launch sequences replayed                   */
  uint64_t particle_steps;  /* of completed jobs                           */
  uint64_t bytes_in_use;
  double busy_s;            /* host time spent waiting on intervals        */
  double wall_s;            /* since creation                              */
  int32_t error;
  int32_t cancelled;        /* jobs cancelled (hd_server_cancel)           */
} hd_server_counters;

int hd_server_create(const hd_server_config* cfg, const hd_device_ctx* ctx, hd_server** out);

/* Queues a job of n_steps > 0 steps; *job_id identifies it.  HD_ENOMEM if the
 * job alone exceeds the budget, HD_EINVAL if it does not fit the slots. */
int hd_server_submit(hd_server* s, const hd_params* params, int64_t n_steps, uint64_t* job_id);

/* *state: 0 queued, 1 running, 2 done, 3 failed, 4 cancelled.  times (may be NULL) gets
 * [submit->admit, submit->done, admit->done] in seconds (-1 if not yet).
 * When done and out != NULL, out is filled like hd_moments. */
int hd_server_poll(hd_server* s, uint64_t job_id, int32_t* state, hd_moment_set* out,
                   double* times);

int hd_server_stats(hd_server* s, hd_server_counters* out);

/* Waits until every submitted job has finished (HD_ESTATE on timeout). */
int hd_server_drain(hd_server* s, double timeout_s);

/* Cancels a job (for callers whose request went away): a queued job leaves
 * the queue at once, a running one is retired after the interval in flight,
 * freeing its slot and budget; either ends in state 4 with no result.
 * Finished jobs are left as they are.  HD_EINVAL for an unknown id. */
int hd_server_cancel(hd_server* s, uint64_t job_id);

/* Stops after the queued and running jobs finish, then releases everything.
 * NULL-safe. */
int hd_server_free(hd_server* s);

/* ---- auxiliary ion swarm (Sec. II.C) ------------------------------------ */

/* The Monte Carlo the paper uses to obtain ion mobilities and
 * momentum-exchange frequencies: ions of one species in a prescribed uniform
 * field E0 collide with a background gas at temperature t_gas_K.  The
 * domain is periodic and the field uniform, so only velocities are
 * followed.  Each step: v_z += e E0 dt / M; then the null-collision test
 * u0 < P_max = 1 - exp(-nu_max dt) with u0 from the stream (seed, tag
 * 3 + 16 f, ion, step); a candidate draws a gas atom from the Maxwellian
 * (two polar pairs of FP64 normal deviates) and collides when u0 <
 * P_max nu(eps)/nu_max at the pair's centre-of-mass energy eps = M_r g^2/(2e)
 * (nu = n_gas k, k linearly interpolated in the table, the last interval
 * beyond its end: counted as overflow); a collision keeps the centre-of-mass
 * velocity and turns the relative velocity to a uniformly random direction
 * (isotropic scattering with Q_m = Q_i + 2 Q_b for He+ in He, Sec. III).
 * Initial velocities: Maxwellian at t_i0_K (stream tag 4 + 16 f, step 0).
 * The mean v_z over the accumulated ion-steps is the drift u; the mobility
 * is u/E0 and Eq (2.6) gives nu = e E0/(M u). */
typedef struct hd_swarm_params {
  int32_t abi_version;     /* must be HD_ABI_VERSION                         */
  int32_t precision;       /* enum hd_precision: ion velocities and collision math */
  int32_t n_fields;        /* independent swarms, one per entry of e0_V_m (>= 1) */
  int32_t n_energy;        /* rate-table points, 2 .. 4096                   */
  int64_t n_ions;          /* ions per swarm; n_fields * n_ions <= 2^31      */
  uint64_t seed;           /* Philox key                                     */
  double n_gas_m3, t_gas_K, m_ion_amu, m_gas_amu;
  double t_i0_K;           /* initial ion temperature                        */
  double dt_s;
  double inv_de_per_eV;    /* table points per eV of centre-of-mass energy   */
  const double* rate_m3_s; /* [n_energy] k(eps_i) = Q_m(eps_i) g(eps_i) at
                              eps_i = i / inv_de_per_eV, g the relative speed
                              with M_r g^2 / (2e) = eps_i [m^3/s];
                              caller-owned, copied                           */
  const double* e0_V_m;    /* [n_fields] field values [V/m]; caller-owned, copied */
} hd_swarm_params;

/* Results of one swarm over the accumulated steps (see hd_swarm_run). */
typedef struct hd_swarm_result {
  double e0_V_m;
  double drift_m_s;        /* mean v_z over ions and accumulated steps       */
  double mean_energy_eV;   /* mean M |v|^2 / (2e)                            */
  double mobility_m2_Vs;   /* drift / E0 (0 for E0 = 0)                      */
  double nu_s;             /* Eq (2.6): e E0 / (M drift) (0 for zero drift)  */
  uint64_t collisions;     /* real collisions since creation                 */
  uint64_t overflow;       /* candidates above the table's last point        */
  int64_t samples;         /* ion-steps in the averages                      */
} hd_swarm_result;

typedef struct hd_swarm hd_swarm;

/* Validates, copies the tables, allocates device state and draws the
 * initial velocities.  Synchronous.  *out is set only on HD_OK. */
int hd_swarm_create(const hd_swarm_params* params, const hd_device_ctx* ctx, hd_swarm** out);

/* Enqueues n_steps >= 0 steps of every ion; with accumulate != 0 each of
 * these steps adds v_z and |v|^2 of every ion to its running sums (the
 * averages of hd_swarm_results).  Returns without waiting. */
int hd_swarm_run(hd_swarm* h, int64_t n_steps, int32_t accumulate);

/* Waits and writes n_fields results (caller-owned array). */
int hd_swarm_results(hd_swarm* h, hd_swarm_result* out);

/* Waits and copies the ions of swarm `field`: velocities (float for HD_FP32,
 * double for HD_FP64) and the running sums of v_z and |v|^2 (double), each
 * array n_ions long (cap >= n_ions); any pointer may be NULL. */
int hd_swarm_get_ions(hd_swarm* h, int32_t field, void* vx, void* vy, void* vz, double* acc_vz,
                      double* acc_v2, int64_t cap);

/* Releases device state.  NULL-safe. */
int hd_swarm_free(hd_swarm* h);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the swarm
 * of hd_swarm_create, hd_swarm_run(n_relax, 0), hd_swarm_run(n_avg, 1) and
 * hd_swarm_results in one call, with the same kernels and the same results,
 * writing n_fields results to the caller-owned host array out.  All device
 * work space (ion velocities and sums, tables, counters) lies in one fixed
 * 64 MiB array inside the library's device code, one per device, held until
 * the process ends: n_fields <= 256 and n_fields * n_ions ions of
 * (3 sizeof(P) + 16) bytes plus the tables must fit (at most 2,396,745
 * FP32 or 1,677,721 FP64 ions in all), else HD_EINVAL names the bytes
 * needed.  No device memory is allocated and no stream is created: the
 * work goes to ctx->stream as given (NULL: the null stream), and the call
 * waits for it.  Calls that overlap on one device share the array and race;
 * each call clears what must start at zero. */
int hd_swarm_run_noalloc(const hd_swarm_params* params, int64_t n_relax, int64_t n_avg,
                         const hd_device_ctx* ctx, hd_swarm_result* out);

/* ---- diagnostics -------------------------------------------------------- */

/* Advances the discharge by n_steps > 0 real steps launched one kernel at a
 * time, with a HIP event pair on the handle's stream around each kernel
 * group, waits, and writes mean device durations in milliseconds to
 * out_ms[0..4]: [0] fused electron step (push, removal, MCC, deposit, and
 * the ion fluid in concurrent workgroups), [1] finalize + field solve,
 * [2] append, [3] compaction + sort (mean over the sorts that ran, 0 if
 * none), [4] whole step.  Used to price the kernels against the roofline. */
int hd_profile_steps(hd_discharge* h, int64_t n_steps, double* out_ms);
/* The same for a batch (every discharge advances by n_steps). */
int hd_batch_profile_steps(hd_batch* b, int64_t n_steps, double* out_ms);

/* Evaluates, on the device, the correctly-rounded primitives the particle
 * arithmetic relies on, for n inputs: out[4k+0] = sqrt(a[k]),
 * out[4k+1] = a[k] / b[k], out[4k+2] = rint(a[k] * 2^32),
 * out[4k+3] = floor(a[k]).  precision selects float or double arrays
 * (a, b, out of the given type, host memory).  Synchronous. */
int hd_diag_arith(int32_t precision, int64_t n, const void* a, const void* b, void* out,
                  const hd_device_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* HD_H */
