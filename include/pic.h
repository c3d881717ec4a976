/*
 * pic.h -- C ABI of the MI355X (gfx950) library for the per-particle step of
 * the 1D3V electrostatic PIC-MCC method of JC-PIC (paper Section 1): field
 * gather from the mesh, Boris push in an imposed magnetic field, move,
 * wall absorption with ion-induced secondary emission, null-collision Monte
 * Carlo against tabulated cross sections, charge deposition, and the 1D
 * Poisson solve between steps.
 *
 * Conventions for every entry point
 *   - Return value: pic_status, 0 = PIC_OK, negative = error.  Argument and
 *     table errors are detected synchronously and leave the state unchanged.
 *   - Host pointers belong to the caller; data is copied during the call and
 *     never retained.  Device buffers belong to the library; they are obtained
 *     through the pic_allocator given to pic_init (hipMalloc when NULL) and
 *     released by pic_free.
 *   - Work is queued on the HIP stream given to pic_init.  pic_step returns as
 *     soon as the work is queued; conditions met on the device (capacity
 *     overflow, non-finite values, a collision frequency above the bound, a
 *     cell out of range) are latched in a flag word and
 *     returned by the next pic_sync or pic_diag.
 *   - A context is used by one host thread at a time.
 *
 * Units: SI, or normalised units when eps0 = 1 and e_unit = 1.  Energies in
 * eV are kinetic energy / e_unit.
 */
#ifndef PIC_H
#define PIC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_MAX_SPECIES 4
#define PIC_MAX_CHAN 8
#define PIC_MAX_BATCH 256

typedef int32_t pic_status;
#define PIC_OK 0
#define PIC_EINVAL (-1)      /* bad argument, table or configuration */
#define PIC_ENOMEM (-2)      /* device or host allocation failed */
#define PIC_EHIP (-3)        /* a HIP runtime call failed */
#define PIC_ECAPACITY (-4)   /* particle or birth capacity exceeded (births dropped) */
#define PIC_ENUMERIC (-5)    /* non-finite particle state */
#define PIC_ESTATE (-6)      /* call not valid in the current state */
#define PIC_ESTALL (-7)      /* reserved: no kernel of the library waits on another workgroup */
#define PIC_ESCRATCH (-8)    /* the work needs more than the fixed scratch of an allocation-free call */

/* Size of the fixed device scratch the allocation-free calls share (one
 * array per GPU the library runs on, held until the process ends). */
#define PIC_NOALLOC_SCRATCH_BYTES (32u << 20)

/* Boundary conditions of the 1D domain [0, L): a column closed on itself
 * (periodic) or a gap between two electrodes (Section 1; Sections 3.5 and
 * 3.6 use the periodic form). */
#define PIC_BC_PERIODIC 0
#define PIC_BC_DIRICHLET 1

/* Collision process kinds (Section 1: tabulated cross sections; Section 3.3:
 * ion charge exchange).  Electron-type kinds act on a projectile against a
 * neutral at rest; ion-type kinds use the relative speed to a neutral drawn
 * from the gas Maxwellian. */
#define PIC_XS_ELASTIC 0      /* isotropic, recoil loss 2m/M (1 - cos chi) */
#define PIC_XS_EXCITATION 1   /* threshold energy removed, isotropic */
#define PIC_XS_IONIZATION 2   /* threshold removed, uniform sharing, e-ion pair born (the ion into species 1; with electrons only, as in a swarm, the ion is not followed) */
#define PIC_XS_ION_CX 3       /* ion takes the neutral's velocity */
#define PIC_XS_ION_ISO 4      /* isotropic scattering in the centre of mass */

/* Particle loading (Section 2: a run starts from the beginning or continues
 * from a stored state). */
#define PIC_LOAD_STRATIFIED 0 /* x_j = (j + u) L / N */
#define PIC_LOAD_RANDOM 1     /* x_j = u L */
#define PIC_LOAD_NONE 2       /* start empty; fill with pic_set_particles */

/* Drive of the electrode at x = 0 (bounded gaps; Sections 3.2 and 3.3).  The
 * electrode and whatever is wired to it form one conductor whose charge per
 * area q changes only by the charge particles bring (absorbed particles
 * bring theirs, each secondary electron emitted takes one away) and by a
 * current source.  Gauss's law at the electrode's surface,
 * q = eps0 E(0) + C (phi0 - V(t)), then fixes its potential phi0; the field
 * is linear in phi0, so phi0 = (C V + q - eps0 E0[psi]) / (C + eps0 / L) with
 * psi the solution for phi0 = 0. */
#define PIC_DRIVE_VOLTAGE 0   /* phi0 = V(t) */
#define PIC_DRIVE_CAPACITOR 1 /* V(t) behind a series capacitor of `cap` F/m^2 (0: a floating electrode);
                                 the DC self-bias develops; starts uncharged, phi0 = V(t) */
#define PIC_DRIVE_CURRENT 2   /* current source J(t) = j_amp sin(2 pi v_freq t + v_phase) A/m^2 into the
                                 electrode; starts at phi0 = 0 */
/* The circuit starts at the first field solve after pic_init, pic_set_particles
 * or pic_load_profiles (new particles); pic_set_circuit then replaces its
 * charge. */
#define PIC_WAVE_SINE 0         /* V(t) = v_amp sin(2 pi v_freq t + v_phase) */
#define PIC_WAVE_TWO_HARMONIC 1 /* V(t) = v_amp [cos(2 pi v_freq t + v_phase) + cos(4 pi v_freq t)] (Section 3.3) */

typedef struct {
    double charge;      /* C (or normalised) */
    double mass;        /* kg */
    double weight;      /* real particles per m^2 per macro-particle */
    int64_t capacity;   /* maximum macro-particles held */
    int64_t n_init;     /* macro-particles loaded by pic_init */
    double vth;         /* sqrt(kT/m) of the loaded Maxwellian, m/s */
    double drift[3];    /* m/s */
    int32_t load;       /* PIC_LOAD_* */
    int32_t pad;
} pic_species_cfg;

/* One discharge (Section 1: gas, pressure, gap, voltage waveform, magnetic
 * field, walls and secondary emission).  Species 0 is the electron species; it
 * receives ionization and secondary electrons.  Species 1, when present, is
 * the ion species; it receives ionization ions and, if its charge is positive,
 * emits secondaries at the walls with probability see_gamma. */
typedef struct {
    int32_t n_cells;        /* mesh cells; nodes at i*dx, dx = length / n_cells */
    int32_t bc;             /* PIC_BC_* */
    int32_t field_solve;    /* 1: Poisson each step; 0: imposed e_ext only */
    int32_t n_species;
    double length, dt, eps0;
    double rho_bg;          /* fixed uniform background charge density */
    double e_unit;          /* charge unit of the eV energy scale */
    double v_amp, v_freq, v_phase;  /* phi(0,t) = v_amp sin(2 pi v_freq t + v_phase), phi(L) = 0 */
    double e_ext[3], b_ext[3];      /* imposed uniform fields */
    double gas_density, gas_temp, gas_mass;  /* m^-3, K, kg */
    double see_gamma, see_temp;     /* secondary yield, emission temperature in eV */
    double perturb_eps;             /* loaded density n0 (1 + eps cos(2 pi m x / L)) */
    int32_t perturb_mode, pad;
    uint64_t seed;                  /* Philox key */
    pic_species_cfg species[PIC_MAX_SPECIES];
    double renew_lz;                /* axial renewal length L_z (m), 0 = off (Section 3.6, after Lafleur,
                                       Baalrud and Chabert): every particle carries its displacement z along
                                       the third axis since injection, z += vz dt; once |z| >= L_z it is
                                       re-injected at the same x with velocities drawn from its species'
                                       initial Maxwellian (vth, drift) and z = 0 */
    int32_t drive;                  /* PIC_DRIVE_*; periodic domains take PIC_DRIVE_VOLTAGE */
    int32_t waveform;               /* PIC_WAVE_* */
    double cap;                     /* series capacitance per area, F/m^2 (PIC_DRIVE_CAPACITOR), >= 0 */
    double j_amp;                   /* current density amplitude, A/m^2 (PIC_DRIVE_CURRENT) */
} pic_config;

typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} pic_allocator;

typedef struct pic_ctx pic_ctx;

/*
 * pic_init: create a context holding n_batch discharges (1 <= n_batch <=
 * PIC_MAX_BATCH) that share n_species and bc, load their particles on the
 * device, deposit, solve the field at t = 0 and take the backward half step
 * v^{-1/2} = Boris(v^0; E^0, B, -dt/2) of the leapfrog start (Section 1:
 * explicit leapfrog).  cfg points to n_batch records.  hip_stream is a
 * hipStream_t (NULL = default stream).  On success *out owns all device
 * memory.
 */
pic_status pic_init(const pic_config* cfg, int32_t n_batch, const pic_allocator* alloc,
                    void* hip_stream, pic_ctx** out);

/*
 * pic_load_xsec: add one collision process for species `species` of discharge
 * `batch` (-1: all discharges) from a table of n >= 2 points (Section 1:
 * tabulated cross sections).  energy_eV must be positive and strictly
 * increasing, sigma_m2 finite and >= 0; values are interpolated linearly in
 * ln(energy), clamped outside the table, and zero below threshold_eV.
 * Processes are tried in the order they were added.  Recomputes the species'
 * maximum collision frequency.  Kinds may not mix electron-type and ion-type
 * within one species; ionization is accepted on species 0 only (its ion goes
 * to species 1 when the context has one).
 */
pic_status pic_load_xsec(pic_ctx* ctx, int32_t batch, int32_t species, int32_t kind,
                         double threshold_eV, int32_t n, const double* energy_eV,
                         const double* sigma_m2);

/*
 * pic_step: queue n_steps >= 0 full steps of every discharge of the
 * context, each the explicit leapfrog step of Section 1 in order: the field
 * gathered at the particles, the Boris push in the imposed magnetic field,
 * the move, walls with absorption and ion-induced secondary emission (or
 * the periodic wrap), collisions by the null-collision method against the
 * tabulated cross sections, births after the survivors, the charge of the
 * particles deposited on the mesh and the field solved at t^{n+1}.  Device
 * conditions (capacity, non-finite state, frequency bound) are latched and
 * reported by the next pic_diag or pic_sync.  n_steps < 0 gives PIC_EINVAL.
 * Asynchronous, on the context's stream.
 */
pic_status pic_step(pic_ctx* ctx, int32_t n_steps);

/*
 * pic_poisson: the field the particles' charge produces on the mesh
 * (Section 1), with the electrode's voltage waveform or drive as the
 * boundary: solve the discharge's 1D Poisson problem at time t_s, in FP64,
 * for the charge density rho_in (host, n_nodes values in C/m^3; NULL: the
 * last deposited density) and copy phi (V) and E (V/m) at the nodes to
 * phi_out / efield_out (host, n_nodes doubles each; either may be NULL).
 * n_nodes = n_cells + 1 for Dirichlet, n_cells for periodic.  Does not change
 * the simulation state.  PIC_EINVAL for a bad batch or a non-finite density.
 * Synchronous.
 */
pic_status pic_poisson(pic_ctx* ctx, int32_t batch, double t_s, const double* rho_in,
                       double* phi_out, double* efield_out);

/* Diagnostic selectors for pic_diag; sizes are for one discharge. */
#define PIC_DIAG_COUNTS 0       /* int64[4 + 2*S]: step, n_nodes, n_species, flags, then per species live count, next_id */
#define PIC_DIAG_RHO 1          /* double[n_nodes]: charge density */
#define PIC_DIAG_PHI 2          /* double[n_nodes] */
#define PIC_DIAG_EFIELD 3       /* double[n_nodes] */
#define PIC_DIAG_DENSITY 4      /* double[S * n_nodes]: number density per species */
#define PIC_DIAG_ENERGY 5       /* double[S + 1]: time-centred kinetic energy per species of the last step, field energy (J/m^2) */
#define PIC_DIAG_WALL 6         /* int64[2*S + 2]: absorbed per species per wall, secondaries emitted per wall */
#define PIC_DIAG_COLL 7         /* int64[S * (3 + PIC_MAX_CHAN)]: candidates, nulls, violations, then per-process counts */
#define PIC_DIAG_NUMAX 8        /* double[2*S]: nu_max per species, then the 32-bit candidate threshold */
#define PIC_DIAG_FLAGS 9        /* int64[1]: latched device flag bits (and clears them) */
#define PIC_DIAG_AVG 10         /* double[1 + (S + 2) * n_nodes]: samples, then mean density per species, mean phi, mean electron energy (eV) */
#define PIC_DIAG_EEPF 11        /* double[2 * PIC_EEPF_BINS + 2]: bulk and wall electron energy histograms, bin width eV, samples */
#define PIC_DIAG_RESET_AVG 12   /* no output: clears the AVG, EEPF, POWER and WALL_EDF accumulators */
#define PIC_DIAG_CHARGE 13      /* double[2]: total charge per unit area on the mesh, and from particle counts */

#define PIC_DIAG_POWER 15       /* double[1 + 5 * S * n_nodes]: samples, then per species the time means of the particle flux density
                                   Gamma = n <vx> (m^-2 s^-1), the x-momentum flux density n <vx^2>, the power density q Gamma E (W/m^3)
                                   that the field (mesh and imposed) gives the species, and two terms of its decomposition (Section 1 names the power
                                   terms; the momentum balance m dGamma/dt + d(m n <vx^2>)/dx = q n E + R times u = Gamma/n): the
                                   inertia term u (m dGamma/dt + d(m Gamma^2/n)/dx) and the pressure term u dp/dx, p =
                                   m (n <vx^2> - Gamma^2/n); the ohmic term is q Gamma E minus both.  dGamma/dt from the previous step's
                                   flux when that step was sampled (else 0); gradients central, one-sided at a wall node
                                   (pic_set_diag; cleared with RESET_AVG) */
#define PIC_DIAG_WALL_ENERGY 16 /* double[2 * S]: kinetic energy carried into each wall (x < 0, x >= L) per species since pic_init, J/m^2
                                   (Section 1: walls; impact energies summed in 2^-20 eV fixed point) */
#define PIC_DIAG_WALL_EDF 17    /* double[S * 2 * PIC_EEPF_BINS + S + 1]: per species and wall (x < 0, x >= L) the
                                   histogram of impact energies since the last reset (bin width emax / PIC_EEPF_BINS,
                                   emax from pic_set_wall_edf), then the bin width (eV) per species, then the samples
                                   of the time averages over the same interval */
#define PIC_DIAG_RENEWED 18     /* int64[S]: axial renewals per species since pic_init */
#define PIC_DIAG_CIRCUIT 19     /* double[2]: potential of the electrode at x = 0 at the last field solve (V),
                                   charge per area of its conductor now (C/m^2; 0 without a circuit) */
#define PIC_DIAG_GRAPHS 20      /* int64[2]: replays of captured step graphs since pic_init, and the steps they ran
                                   (the other steps were launched directly) */
#define PIC_DIAG_TIMING 14      /* double[6]: finalize launches, finalize ms, push launches, push ms, events launches, events ms
                                   (pic_profile; one launch of each kernel covers every species) */

#define PIC_EEPF_BINS 256
#define PIC_WINDOW_RING 64      /* completed RF windows kept per discharge (pic_get_windows) */

/*
 * pic_diag: the engine's diagnostics (Section 1 lists density, potential
 * and field profiles, energies, electron energy distributions, wall fluxes
 * and collision statistics; the selectors above say each layout).
 * Synchronise the stream, then copy diagnostic `what` of discharge `batch`
 * into out (host, out_bytes bytes, owned by the caller).  Returns PIC_EINVAL
 * for an unknown selector or batch or if out_bytes is too small, and any
 * latched device error (after copying).
 */
pic_status pic_diag(pic_ctx* ctx, int32_t batch, int32_t what, void* out, size_t out_bytes);

/*
 * pic_get_particles: copy the n (<= cap) particles of one species and
 * discharge in their canonical order (Section 1: a paused run can be resumed):
 * cell index, in-cell offset in [0,1), velocity, id.  *n_out receives the count
 * and *next_id the next id the species will assign.  The canonical order is
 * the survivors of every step in their previous order followed by that step's
 * births in the order of their parents.  When particle arrays are requested
 * and absorbed particles still leave holes, the context is compacted first
 * (the order is unchanged).  Synchronous.
 */
pic_status pic_get_particles(pic_ctx* ctx, int32_t batch, int32_t species, int64_t cap,
                             int32_t* cell, float* off, float* vx, float* vy, float* vz,
                             uint32_t* id, int64_t* n_out, uint32_t* next_id);

/*
 * pic_set_particles: replace the particles of one species and discharge
 * (n <= capacity), set the step index of the whole context to `step` and the
 * species' next id, then re-deposit and re-solve the field of that discharge
 * at t = step * dt.  Positions are cell in [0, n_cells) and off in [0,1).
 * Non-finite velocities give PIC_ENUMERIC.  Synchronous.
 */
pic_status pic_set_particles(pic_ctx* ctx, int32_t batch, int32_t species, int64_t n,
                             const int32_t* cell, const float* off, const float* vx,
                             const float* vy, const float* vz, const uint32_t* id,
                             uint32_t next_id, uint64_t step);

/*
 * pic_load_profiles: restart discharge `batch` from profiles (a warm start;
 * Section 1 loads particles into the mesh at the start of a run).  For every
 * species s, n[s] particles are drawn from the density profile
 * density[s * m + i] and the temperature profile temp_eV[s * m + i], both
 * given at the m points x_i = i L / (m - 1) (2 <= m <= 4097) and linear in
 * between: positions x_j = F^-1((j + u_j) / n[s]) with F the integral of the
 * density divided by its total (a uniform profile gives the stratified load),
 * velocities Maxwellian at the local temperature (scale sqrt(e T / m_s)),
 * ids 0 .. n[s] - 1 and next id n[s].  Then the charge is deposited, the field
 * solved at the discharge's current time and the velocities moved back half
 * a step, as at pic_init.  Density values are relative (any positive scale);
 * negative or non-finite values, a zero total with n[s] > 0, or n[s] above
 * the capacity give PIC_EINVAL with no state change.  Synchronous.
 */
pic_status pic_load_profiles(pic_ctx* ctx, int32_t batch, int32_t m, const double* density,
                             const double* temp_eV, const int64_t* n);

/*
 * pic_get_axial / pic_set_axial: the axial displacements z (m) of the
 * particles of one species and discharge, in canonical order (one per
 * particle of pic_get_particles), when the context renews particles
 * (renew_lz > 0; Section 3.6).  pic_set_particles and pic_load_profiles set
 * z = 0; pic_set_axial then replaces them (n must equal the species' count).
 * PIC_EINVAL without renewal, for a size mismatch, or a non-finite value.
 * get: *n_out receives the count; with cap below it (or z NULL) nothing is
 * copied.  Synchronous.
 */
pic_status pic_get_axial(pic_ctx* ctx, int32_t batch, int32_t species, int64_t cap, double* z, int64_t* n_out);
pic_status pic_set_axial(pic_ctx* ctx, int32_t batch, int32_t species, int64_t n, const double* z);

/*
 * pic_set_circuit: replace the charge per area q of the driven electrode's
 * conductor of discharge `batch` (PIC_DRIVE_CAPACITOR or PIC_DRIVE_CURRENT;
 * e.g. when resuming a run) and re-solve that discharge's field.  PIC_EINVAL
 * without a circuit or for a non-finite q.  Synchronous.
 */
pic_status pic_set_circuit(pic_ctx* ctx, int32_t batch, double q);

/*
 * pic_set_windows: close a time-averaging window of discharge `batch` every
 * `steps` steps from its current step (steps = 0: off).  At the end of each
 * window the step itself moves the window's sums (the PIC_DIAG_AVG
 * accumulators: densities, potential, electron energy) into a ring of
 * PIC_WINDOW_RING completed windows on the device and restarts them, so a
 * batch of discharges with different RF periods needs no host
 * synchronisation per window (Section 1: periodic steady states are judged
 * on RF-period averages).  Needs pic_set_diag enabled.  PIC_EINVAL for
 * steps < 0.  Synchronous.
 *
 * pic_get_windows: copies the completed windows first .. first + count - 1
 * of discharge `batch` to out, each 1 + (S + 2) n_nodes doubles in the
 * layout of PIC_DIAG_AVG (samples, mean densities, mean potential, electron
 * mean energy), and sets *n_done to the number of windows completed so far.
 * count may be 0 (query).  PIC_EINVAL when a requested window is not
 * completed yet or already overwritten (first < n_done - PIC_WINDOW_RING).
 * Synchronous.
 */
pic_status pic_set_windows(pic_ctx* ctx, int32_t batch, int64_t steps);
pic_status pic_get_windows(pic_ctx* ctx, int32_t batch, int64_t first, int32_t count, double* out,
                           int64_t* n_done);

/* pic_sync: wait for queued work; return a latched device error if any. */
pic_status pic_sync(pic_ctx* ctx);

/* pic_strerror: static text for a status. */
const char* pic_strerror(pic_status s);

/* pic_free: wait for queued work and release every buffer. */
void pic_free(pic_ctx* ctx);

/* pic_set_diag: when enable is non-zero, every step also accumulates the
 * time averages of the densities, the potential and the electron mean energy
 * (PIC_DIAG_AVG), and electron energy histograms of bin width
 * eepf_emax_eV / PIC_EEPF_BINS in the bulk (middle tenth of a bounded gap,
 * whole domain when periodic) and at the walls (PIC_DIAG_EEPF) (Section 1:
 * density and potential profiles, electron energy probability functions in
 * the bulk and at the walls).  Samples are taken on the state at the end of
 * each step (velocities after collisions, the step's births included); the
 * mean energy at a node is sum(n eps) / sum(n) over the samples, with the
 * linear weights of the charge deposit.  Species 0 is taken as the electrons.
 * PIC_EINVAL when eepf_emax_eV is not positive and finite. */
pic_status pic_set_diag(pic_ctx* ctx, int32_t enable, double eepf_emax_eV);

/* pic_set_wall_edf: energy range [0, emax_eV) of the histogram of the impact
 * energies m |v|^2 / 2e of species `species` at each wall (PIC_DIAG_WALL_EDF;
 * Section 1: wall diagnostics; for ions the ion flux-energy distribution at
 * the electrodes), for every discharge of the context.  Defaults: 64 eV for
 * species 0, 1024 eV for the others.  The histograms fill while pic_set_diag
 * is enabled.  PIC_EINVAL for a species out of range or emax_eV not positive
 * and finite.  Synchronous (waits for queued work). */
pic_status pic_set_wall_edf(pic_ctx* ctx, int32_t species, double emax_eV);

/* pic_profile: when enable is non-zero, pic_step records a pair of HIP
 * events on the context's stream around every kernel it launches and
 * accumulates their elapsed times (read with PIC_DIAG_TIMING); enabling
 * clears the sums.  A measuring aid; it adds two event records per launch. */
pic_status pic_profile(pic_ctx* ctx, int32_t enable);

/* pic_retire: a retired discharge (retired != 0) is skipped by pic_step and
 * keeps its state; a batched sweep retires discharges as they converge.
 * Synchronous. */
pic_status pic_retire(pic_ctx* ctx, int32_t batch, int32_t retired);

/* pic_sort: queue a stable sort of every species of every discharge by cell
 * index (particles with equal cells keep their order).  pic_config_tiles can
 * make pic_step do this every K steps.  The canonical order changes, and
 * with it the ids later births receive (in their parents' order): a run with
 * births then draws other random numbers than an unsorted run.
 * Asynchronous. */
pic_status pic_sort(pic_ctx* ctx);

/* pic_thin: population control of a species over every running discharge of
 * the context, for the swarm setting of Section 4, where ionization makes an
 * electron swarm grow without bound: where `species` holds more than `above`
 * live particles, each is kept with probability keep / live, by an integer
 * test on a Philox draw keyed by the particle's id and the step (call 7), and
 * the removed ones are compacted away at once.  The survivors keep their
 * order and ids (next_id is unchanged), so every per-particle average is
 * unbiased; the kept count is keep on average, not exactly.  PIC_EINVAL for
 * a species out of range, keep < 0 or keep > above.  Asynchronous, on the
 * context's stream; call it between steps. */
pic_status pic_thin(pic_ctx* ctx, int32_t species, int64_t above, int64_t keep);

/* pic_sort_noalloc: pic_sort for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result, with their scratch (the
 * per-tile cell histogram and the group sums) in a fixed device array of
 * PIC_NOALLOC_SCRATCH_BYTES per GPU, resolved at pic_init, instead of the
 * buffer pic_sort allocates at its first call.  Calls no allocating routine.
 * Needs (tiles x cells + discharges x 64 x cells) x 4 bytes, tiles being the
 * capacity of the largest species over 1024 (for example one species of up
 * to 8.1e6 particles on 1024 cells); larger contexts get PIC_ESCRATCH with no
 * work queued.  Every allocation-free call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (on different streams, or from different
 * threads) race.  Asynchronous, on the context's stream. */
pic_status pic_sort_noalloc(pic_ctx* ctx);

/* pic_use_graphs: when enable is non-zero (the default), pic_step captures a
 * chunk of consecutive steps once into a HIP graph on a private stream and
 * replays it on the context's stream, which removes the host launch gaps
 * between kernels; all per-step state lives on the device, so one capture
 * serves any number of steps.  The chunk is the least multiple of 32 steps
 * that the sort and compaction intervals divide (graphs are not used when
 * that exceeds 1024 steps); steps short of a whole chunk are launched
 * directly.  PIC_DIAG_GRAPHS counts the replays.  Profiling (pic_profile)
 * uses direct launches. */
pic_status pic_use_graphs(pic_ctx* ctx, int32_t enable);

/* pic_config_events: where the step's events (collision candidates, axial
 * renewals, ions absorbed at an emitting wall: the few particles per step
 * that need the null-collision Monte Carlo of Section 1, the renewal or
 * the secondary emission) are processed.  in_push = 0 (the default): one
 * events kernel after the push, its waves packed over all events of the
 * step.  in_push = 1: each push workgroup processes the events of its own
 * tiles after its push, with no further launch, which shortens the step of
 * a workload too small to fill the GPU; this applies to tiles of 256
 * threads with one to four particles each (other shapes keep the events
 * kernel).  The results are the same
 * either way, bit for bit.  PIC_EINVAL for another value.  Synchronous;
 * takes effect at the next pic_step. */
pic_status pic_config_events(pic_ctx* ctx, int32_t in_push);

/* pic_config_tiles: tile shape of the particle kernels (particles per thread
 * 1, 2, 4 or 8; threads per workgroup 256, 512 or 1024; the nearest built
 * shape is used: 1024 threads take four particles each, 512 four or, in
 * the general kernel, eight), the interval in steps of the sort by cell (0 = never) and
 * the interval in steps of the compaction that removes the holes absorbed
 * particles leave (1 .. 1024, default 16; bounded runs only).  With graphs,
 * the replayed chunk is the least multiple of 32 steps both intervals
 * divide.  Takes effect at the next pic_step. */
pic_status pic_config_tiles(pic_ctx* ctx, int32_t particles_per_thread,
                            int32_t threads_per_group, int32_t sort_every, int32_t compact_every);

#ifdef __cplusplus
}
#endif
#endif
