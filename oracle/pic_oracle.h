/*
 * pic_oracle.h -- plain FP64 CPU oracle of the 1D3V electrostatic PIC-MCC
 * step (explicit leapfrog, Boris push, null-collision Monte Carlo against
 * tabulated cross sections, walls with ion-induced secondary emission, and
 * the 1D Poisson solve on the mesh; paper Section 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant with the GPU library; the two meet only through
 * the seeded workload records and the published Philox4x32-10 definition that
 * each side implements on its own.
 *
 * Particles are held at absolute FP64 positions x in [0, L) with FP64
 * velocities and 32-bit ids.  Everything is sequential and in the order the
 * method states, so that it can be checked by eye.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_SPECIES 4
#define ORC_MAX_CHAN 8
#define ORC_EEPF_BINS 256

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ECAPACITY = -4,
       ORC_ENUMERIC = -5, ORC_ESTATE = -6 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_DIRICHLET = 1 };
enum { ORC_XS_ELASTIC = 0, ORC_XS_EXCITATION = 1, ORC_XS_IONIZATION = 2,
       ORC_XS_ION_CX = 3, ORC_XS_ION_ISO = 4 };
enum { ORC_LOAD_STRATIFIED = 0, ORC_LOAD_RANDOM = 1, ORC_LOAD_NONE = 2 };
/* drive of the electrode at x = 0 (bounded domains) */
enum { ORC_DRIVE_VOLTAGE = 0, ORC_DRIVE_CAPACITOR = 1, ORC_DRIVE_CURRENT = 2 };
/* source waveform: sine V sin(2 pi f t + phase); two harmonics
 * V [cos(2 pi f t + phase) + cos(4 pi f t)] */
enum { ORC_WAVE_SINE = 0, ORC_WAVE_TWO_HARMONIC = 1 };

typedef struct {
    double charge, mass, weight;      /* C, kg, real particles per m^2 per macro */
    int64_t capacity, n_init;
    double vth;                       /* sqrt(kT/m) of the loaded Maxwellian */
    double drift[3];
    int32_t load, pad;
} orc_species;

typedef struct {
    int32_t n_cells, bc, field_solve, n_species;
    double length, dt, eps0, rho_bg, e_unit;
    double v_amp, v_freq, v_phase;
    double e_ext[3], b_ext[3];
    double gas_density, gas_temp, gas_mass;
    double see_gamma, see_temp;
    double perturb_eps;
    int32_t perturb_mode, pad;
    uint64_t seed;
    orc_species sp[ORC_MAX_SPECIES];
    double renew_lz;                  /* axial renewal length (m); 0: no renewal */
    int32_t drive, waveform;          /* ORC_DRIVE_*, ORC_WAVE_* */
    double cap;                       /* series capacitance per area (F/m^2), capacitor drive */
    double j_amp;                     /* current density amplitude (A/m^2), current drive */
} orc_config;

/* Counters of one run: event counts (integer-exact) and the kinetic energy
 * carried into each wall (J per m^2 of electrode). */
typedef struct {
    int64_t absorbed[ORC_MAX_SPECIES][2];   /* [species][wall 0 = x<0, 1 = x>=L] */
    int64_t see_emitted[2];
    int64_t candidates[ORC_MAX_SPECIES];
    int64_t nulls[ORC_MAX_SPECIES];
    int64_t coll[ORC_MAX_SPECIES][ORC_MAX_CHAN];
    int64_t violations[ORC_MAX_SPECIES];
    int64_t dropped;
    double wall_energy[ORC_MAX_SPECIES][2];  /* [species][wall]: sum of m w |v|^2 / 2 at impact */
    int64_t renewed[ORC_MAX_SPECIES];        /* axial renewals */
} orc_counters;

typedef struct orc_sim orc_sim;

int  orc_create(const orc_config* cfg, orc_sim** out);
void orc_free(orc_sim* s);
int  orc_load_xsec(orc_sim* s, int32_t species, int32_t kind, double threshold_eV,
                   int32_t n, const double* energy_eV, const double* sigma_m2);
/* Load particles (Philox draws at step 0xFFFFFFFF), deposit, solve at t = 0,
 * and take the backward half step of the leapfrog start. */
int  orc_load(orc_sim* s);
/* velocity moments of species k at the nodes (flux and x-momentum flux densities) */
int  orc_get_moments(const orc_sim* s, int32_t k, double* flux, double* mom);
/* start from density and temperature profiles at m points over [0, L]
 * (arrays [n_species][m]); n[k] particles of species k */
int  orc_load_profiles(orc_sim* s, int32_t m, const double* density, const double* temp_ev,
                       const int64_t* n);
/* Replace species state; positions in [0, L). */
int  orc_set_particles(orc_sim* s, int32_t species, int64_t n, const double* x,
                       const double* vx, const double* vy, const double* vz,
                       const uint32_t* id, uint32_t next_id);
int  orc_set_axial(orc_sim* s, int32_t species, int64_t n, const double* z);
int  orc_get_axial(const orc_sim* s, int32_t species, int64_t cap, double* z);
int  orc_get_particles(const orc_sim* s, int32_t species, int64_t cap, double* x,
                       double* vx, double* vy, double* vz, uint32_t* id, int64_t* n,
                       uint32_t* next_id);
int  orc_set_step(orc_sim* s, uint64_t step);
/* External circuit of the electrode at x = 0: out[0] = its potential at the
 * last solve, out[1] = q, the charge per area on the electrode's conductor
 * (its surface facing the plasma plus the series capacitor's plate).  Set:
 * replaces q (e.g. on resume). */
int  orc_get_circuit(const orc_sim* s, double out[2]);
int  orc_set_circuit(orc_sim* s, double q);
uint64_t orc_get_step(const orc_sim* s);
/* Deposit the current particles and solve the field at t = step*dt. */
int  orc_refresh_field(orc_sim* s);
int  orc_step(orc_sim* s, int32_t n_steps);
/* Standalone field solve of the mesh problem for charge density rho_in
 * (n_nodes values) at time t; phi_out / e_out may be NULL. */
int  orc_poisson(const orc_sim* s, double t, const double* rho_in, double* phi_out,
                 double* e_out);
int  orc_n_nodes(const orc_sim* s);
int  orc_get_field(const orc_sim* s, double* rho, double* phi, double* efield);
int  orc_get_density(const orc_sim* s, int32_t species, double* dens);
int  orc_get_counters(const orc_sim* s, orc_counters* out);
/* 0 (the default): the sequential step; n > 0: the parallel step on n OpenMP
 * threads (fixed chunks of particles merged in chunk order: the same result
 * for every n; only the order of the floating-point sums of the deposit,
 * the kinetic energy, the wall energies and the sampled energy profile
 * differs from the sequential step). */
int  orc_set_threads(orc_sim* s, int32_t threads);
/* Time means (since the last reset) of species k's power terms at the
 * nodes, [5][n_nodes]: flux Gamma, x-momentum flux n <vx^2>, q Gamma E, the
 * inertia term and the pressure term (the ohmic term is q Gamma E minus
 * both). */
int  orc_get_power(const orc_sim* s, int32_t k, double* out);
/* Kinetic energy of each species at the last step (time-centred), field energy. */
int  orc_get_energy(const orc_sim* s, double* ke_species, double* fe);
int  orc_get_numax(const orc_sim* s, int32_t species, double* numax, uint32_t* t32);

/* Time-accumulated diagnostics, sampled at the end of every step while
 * enabled: mean density per species, mean potential and the electron mean
 * energy at the nodes; electron energy histograms of the bulk cells and of
 * the wall impacts over [0, eepf_emax); per species and wall, the histogram
 * of impact energies over [0, emax_k) (64 eV for species 0, 1024 eV for the
 * others unless set).  Layouts:
 *   avg:      [samples, density[S][nn], phi[nn], mean electron energy (eV)[nn]]
 *   eepf:     [bulk[BINS], wall[BINS], bin width (eV), samples]
 *   wall edf: [counts[S][2][BINS], bin width per species (eV)[S], samples] */
int  orc_set_diag(orc_sim* s, int32_t enable, double eepf_emax_ev);
int  orc_set_wall_edf(orc_sim* s, int32_t species, double emax_ev);
int  orc_reset_avg(orc_sim* s);
int  orc_get_avg(const orc_sim* s, double* out);
int  orc_get_eepf(const orc_sim* s, double* out);
int  orc_get_wall_edf(const orc_sim* s, double* out);

/* Building blocks exposed for the pins. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t x);
void orc_boris(double v[3], const double e[3], const double b[3], double qm, double h);
void orc_rotate(const double d[3], double cos_chi, double phi, double out[3]);

#ifdef __cplusplus
}
#endif
#endif
