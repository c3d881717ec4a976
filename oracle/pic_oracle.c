/*
 * pic_oracle.c -- plain FP64 CPU oracle of the 1D3V electrostatic PIC-MCC
 * method (paper Section 1: explicit leapfrog, Boris pusher, null-collision
 * Monte Carlo, tabulated cross sections, walls and secondary emission, the
 * field computed on a mesh from the particles' own charge).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.
 *
 * The paper fixes the scheme but none of its numerical details; every reading
 * taken here is stated where it is used (linear cloud-in-cell weighting, wall
 * nodes of half volume, Gauss's law at the walls, isotropic scattering with
 * the Vahedi-Surendra rotation, uniform ionization energy sharing, charge
 * exchange with a thermal neutral, a half-Maxwellian flux for secondaries,
 * Philox4x32-10 keyed by (seed, particle id, step)).
 *
 * Plain loops, FP64 throughout.  Sequential by default; orc_set_threads
 * selects a parallel step (OpenMP over fixed chunks of particles, merged in
 * chunk order) whose result does not depend on the thread count, for timing
 * on the host's cores and for long statistical runs.
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define K_B 1.380649e-23
#define TWO_PI 6.283185307179586476925286766559

typedef struct {
    double *x, *vx, *vy, *vz;
    double* z;                        /* virtual axial displacement since the last renewal */
    uint32_t* id;
    int64_t n, cap;
    uint32_t next_id;
} pop_t;

typedef struct {
    int32_t kind;
    double th;
    int32_t n;
    double *e, *s;
} chan_t;

typedef struct {          /* a particle waiting to be appended after the sweep */
    double x, vx, vy, vz;
} birth_t;

typedef struct {
    birth_t* b;
    int64_t n, cap;
} blist_t;

/* What a run of particles of one species adds in a step: counters, births
 * (in the order they are made), the kinetic-energy sum, and the wall-impact
 * histograms of the diagnostics.  The sequential step has one run per
 * species; the parallel step one per chunk of ORC_CHUNK particles, merged in
 * chunk order, so that its result does not depend on the thread count. */
typedef struct {
    orc_counters cnt;
    blist_t births[ORC_MAX_SPECIES];
    double ke;
    int64_t eepf_wall[ORC_EEPF_BINS];  /* electrons: wall-impact energies */
    int64_t wedf[2][ORC_EEPF_BINS];    /* this species: impact energies at each wall */
    int64_t keep;                      /* survivors of the run */
    int rc;                            /* first error of the run */
} sink_t;

#define ORC_CHUNK 4096

struct orc_sim {
    orc_config c;
    double dx;
    int32_t nn;                       /* mesh nodes */
    pop_t p[ORC_MAX_SPECIES];
    chan_t ch[ORC_MAX_SPECIES][ORC_MAX_CHAN];
    int32_t nch[ORC_MAX_SPECIES];
    double numax[ORC_MAX_SPECIES];
    uint32_t t32[ORC_MAX_SPECIES];
    double *rho, *phi, *ef;
    double* sum[ORC_MAX_SPECIES];     /* weight sums per node */
    double* dens[ORC_MAX_SPECIES];
    uint64_t step;
    orc_counters cnt;
    /* external circuit: the conductor's charge is qbase + the source's charge
     * since t = 0 + the charge collected from particles since the start */
    double qbase;
    int32_t circ_init;
    double ke[ORC_MAX_SPECIES], fe;
    blist_t births[ORC_MAX_SPECIES];
    /* the parallel step (threads > 0): its chunk runs, a second population to
     * compact into, and per-chunk partial sums of the deposit */
    int32_t threads;
    sink_t* runs;
    int64_t nruns;
    pop_t spare[ORC_MAX_SPECIES];
    double* part;
    int64_t npart;
    /* time-accumulated diagnostics, sampled after every step while enabled */
    int32_t diag;
    double eepf_emax, wedf_emax[ORC_MAX_SPECIES];
    double* av_dens[ORC_MAX_SPECIES];  /* sum over samples of the density per node */
    double *av_phi, *av_neps;         /* potential; electron density times energy (eV) */
    double av_samples;
    int64_t eepf[2][ORC_EEPF_BINS];   /* electrons: bulk cells, wall impacts */
    /* power decomposition: per species the time sums of flux, x-momentum
     * flux, q Gamma E, inertia and pressure terms; the last sampled flux */
    double* av_pw[ORC_MAX_SPECIES];    /* [5][nn] */
    double* gprev[ORC_MAX_SPECIES];
    double* pw_tmp;                    /* [4][nn]: Gamma, n <vx^2>, m Gamma^2 / n, p */
    uint64_t pw_next;                  /* the step whose previous flux is stored (else none) */
    int64_t wedf[ORC_MAX_SPECIES][2][ORC_EEPF_BINS];
};

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
 * multiply-xor round function on a 128-bit counter, the 64-bit key bumped by
 * the Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from the top 23 bits: an odd multiple of 2^-24, exact in
 * both binary32 and binary64, never 0 or 1. */
double orc_u01(uint32_t x)
{
    return (double)(((x >> 9) << 1) | 1u) * (1.0 / 16777216.0);
}

static void draw(const orc_sim* s, uint32_t id, uint32_t step, int32_t species,
                 uint32_t call, uint32_t out[4])
{
    uint32_t ctr[4] = {id, step, ((uint32_t)species << 24) | call, 0u};
    uint32_t key[2] = {(uint32_t)(s->c.seed & 0xffffffffu), (uint32_t)(s->c.seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Box-Muller: two standard normals from two uniforms. */
static void box_muller(double ua, double ub, double* g0, double* g1)
{
    double r = sqrt(-2.0 * log(ua));
    *g0 = r * cos(TWO_PI * ub);
    *g1 = r * sin(TWO_PI * ub);
}

/* ------------------------------------------------------------------------ */
/* Boris push over a time h: half electric kick, magnetic rotation with
 * t = (q/m) B h/2 and s = 2t/(1+|t|^2), half electric kick. */
void orc_boris(double v[3], const double e[3], const double b[3], double qm, double h)
{
    double a = 0.5 * qm * h;
    double vm[3] = {v[0] + a * e[0], v[1] + a * e[1], v[2] + a * e[2]};
    double t[3] = {a * b[0], a * b[1], a * b[2]};
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double sf = 2.0 / (1.0 + t2);
    double sv[3] = {sf * t[0], sf * t[1], sf * t[2]};
    double vp[3] = {vm[0] + (vm[1] * t[2] - vm[2] * t[1]),
                    vm[1] + (vm[2] * t[0] - vm[0] * t[2]),
                    vm[2] + (vm[0] * t[1] - vm[1] * t[0])};
    double vq[3] = {vm[0] + (vp[1] * sv[2] - vp[2] * sv[1]),
                    vm[1] + (vp[2] * sv[0] - vp[0] * sv[2]),
                    vm[2] + (vp[0] * sv[1] - vp[1] * sv[0])};
    v[0] = vq[0] + a * e[0];
    v[1] = vq[1] + a * e[1];
    v[2] = vq[2] + a * e[2];
}

/* New direction after scattering by polar angle chi and azimuth phi about the
 * incident unit direction d (Vahedi & Surendra 1995 form, reference axis x;
 * when d is within 1e-6 of the x axis the y axis is used instead). */
void orc_rotate(const double d[3], double cos_chi, double phi, double out[3])
{
    double sin_chi = sqrt(fmax(0.0, 1.0 - cos_chi * cos_chi));
    double cp = cos(phi), sp = sin(phi);
    double a, b, c;                          /* components in the rotated frame */
    int alt;
    double ct = d[0];
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    if (st > 1e-6) {
        a = d[0]; b = d[1]; c = d[2];
        alt = 0;
    } else {                                  /* cyclic relabel (y, z, x) */
        a = d[1]; b = d[2]; c = d[0];
        ct = a;
        st = sqrt(fmax(0.0, 1.0 - ct * ct));
        alt = 1;
    }
    double A = sin_chi / st;
    double na = a * cos_chi + sin_chi * cp * st;
    double nb = b * cos_chi + A * (sp * c - cp * a * b);
    double nc = c * cos_chi - A * (sp * b + cp * a * c);
    if (!alt) {
        out[0] = na; out[1] = nb; out[2] = nc;
    } else {
        out[1] = na; out[2] = nb; out[0] = nc;
    }
}

/* ------------------------------------------------------------------------ */
static int is_periodic(const orc_sim* s) { return s->c.bc == ORC_BC_PERIODIC; }

static double node_volume(const orc_sim* s, int i)
{
    if (!is_periodic(s) && (i == 0 || i == s->nn - 1)) return 0.5 * s->dx;
    return s->dx;
}

/* Cell and in-cell fraction of position x (linear cloud-in-cell weighting,
 * nodes at i*dx). */
static void locate(const orc_sim* s, double x, int64_t* c, int64_t* c1, double* f)
{
    int64_t nc = s->c.n_cells;
    double xi = x / s->dx;
    int64_t k = (int64_t)floor(xi);
    double fr = xi - (double)k;
    if (is_periodic(s)) {
        if (k >= nc) { k -= nc; }
        if (k < 0) { k += nc; }
        *c = k;
        *c1 = (k + 1 == nc) ? 0 : k + 1;
    } else {
        if (k >= nc) { k = nc - 1; fr = 1.0; }
        if (k < 0) { k = 0; fr = 0.0; }
        *c = k;
        *c1 = k + 1;
    }
    *f = fr;
}

static double gather(const orc_sim* s, double x)
{
    int64_t c, c1;
    double f;
    locate(s, x, &c, &c1, &f);
    return (1.0 - f) * s->ef[c] + f * s->ef[c1];
}

/* The source waveform (Section 3.3 gives the two-harmonic form). */
static double source(const orc_sim* s, double t)
{
    double w = TWO_PI * s->c.v_freq;
    if (s->c.waveform == ORC_WAVE_TWO_HARMONIC)
        return s->c.v_amp * (cos(w * t + s->c.v_phase) + cos(2.0 * w * t));
    return s->c.v_amp * sin(w * t + s->c.v_phase);
}

static double voltage(const orc_sim* s, double t)
{
    if (is_periodic(s)) return 0.0;
    return source(s, t);
}

static int circuit_mode(const orc_sim* s)
{
    return !is_periodic(s) && s->c.field_solve && s->c.drive != ORC_DRIVE_VOLTAGE;
}

/* Charge per area the particles have brought to the electrode at x = 0 since
 * the start: absorbed particles bring their charge, each secondary electron
 * it emits takes an electron's charge away. */
static double q_collected(const orc_sim* s)
{
    double q = 0.0;
    for (int k = 0; k < s->c.n_species; ++k)
        q += s->c.sp[k].charge * s->c.sp[k].weight * (double)s->cnt.absorbed[k][0];
    q -= s->c.sp[0].charge * s->c.sp[0].weight * (double)s->cnt.see_emitted[0];
    return q;
}

/* Charge per area the current source has delivered since t = 0:
 * integral of j_amp sin(w t + phase). */
static double q_source(const orc_sim* s, double t)
{
    if (s->c.drive != ORC_DRIVE_CURRENT) return 0.0;
    double w = TWO_PI * s->c.v_freq;
    return s->c.j_amp / w * (cos(s->c.v_phase) - cos(w * t + s->c.v_phase));
}

/* ------------------------------------------------------------------------ */
/* Cross sections: linear interpolation in ln(eps), clamped to the end values
 * outside the table, zero below the channel threshold. */
static double sigma_at(const chan_t* ch, double eps)
{
    if (eps < ch->th) return 0.0;
    if (eps <= ch->e[0]) return ch->s[0];
    if (eps >= ch->e[ch->n - 1]) return ch->s[ch->n - 1];
    int lo = 0, hi = ch->n - 1;            /* e[lo] <= eps < e[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (ch->e[mid] <= eps) lo = mid; else hi = mid;
    }
    double t = (log(eps) - log(ch->e[lo])) / (log(ch->e[hi]) - log(ch->e[lo]));
    return ch->s[lo] + t * (ch->s[hi] - ch->s[lo]);
}

static int electron_kind(int kind)
{
    return kind == ORC_XS_ELASTIC || kind == ORC_XS_EXCITATION || kind == ORC_XS_IONIZATION;
}

/* Maximum collision frequency of a species and the 32-bit candidate threshold
 * T32 = floor(P_null 2^32), P_null = 1 - exp(-nu_max dt).  Electron-type
 * projectiles: 1.05 x the maximum of n_g sum_k sigma_k(eps) v(eps) over a
 * log-uniform grid ten times finer than the longest table.  Ion-type
 * projectiles: n_g max(sum_k sigma_k) g_max, g_max the relative speed of a
 * projectile at the top table energy plus six neutral thermal speeds. */
static void update_numax(orc_sim* s, int sp)
{
    int nch = s->nch[sp];
    if (nch == 0) { s->numax[sp] = 0.0; s->t32[sp] = 0; return; }
    double elo = s->ch[sp][0].e[0], ehi = s->ch[sp][0].e[s->ch[sp][0].n - 1];
    int nmax = 0;
    for (int k = 0; k < nch; ++k) {
        if (s->ch[sp][k].e[0] < elo) elo = s->ch[sp][k].e[0];
        if (s->ch[sp][k].e[s->ch[sp][k].n - 1] > ehi) ehi = s->ch[sp][k].e[s->ch[sp][k].n - 1];
        if (s->ch[sp][k].n > nmax) nmax = s->ch[sp][k].n;
    }
    int m = 10 * nmax;
    double lelo = log(elo), lehi = log(ehi);
    double mass = s->c.sp[sp].mass, ng = s->c.gas_density;
    double best = 0.0;
    int ion = !electron_kind(s->ch[sp][0].kind);
    for (int j = 0; j < m; ++j) {
        double eps = exp(lelo + (double)j * (lehi - lelo) / (double)(m - 1));
        double sig = 0.0;
        for (int k = 0; k < nch; ++k) sig += sigma_at(&s->ch[sp][k], eps);
        double val = ion ? sig : ng * sig * sqrt(2.0 * s->c.e_unit * eps / mass);
        if (val > best) best = val;
    }
    double numax;
    if (ion) {
        double gmax = sqrt(2.0 * s->c.e_unit * ehi / mass) +
                      6.0 * sqrt(K_B * s->c.gas_temp / s->c.gas_mass);
        numax = ng * best * gmax;
    } else {
        numax = 1.05 * best;
    }
    double pnull = 1.0 - exp(-numax * s->c.dt);
    double t = floor(pnull * 4294967296.0);
    if (t > 4294967295.0) t = 4294967295.0;
    s->numax[sp] = numax;
    s->t32[sp] = (uint32_t)t;
}

/* ------------------------------------------------------------------------ */
static int pop_alloc(pop_t* p, int64_t cap)
{
    p->cap = cap;
    p->n = 0;
    p->next_id = 0;
    size_t n = (size_t)(cap > 0 ? cap : 1);
    p->x = calloc(n, sizeof(double));
    p->vx = calloc(n, sizeof(double));
    p->vy = calloc(n, sizeof(double));
    p->vz = calloc(n, sizeof(double));
    p->z = calloc(n, sizeof(double));
    p->id = calloc(n, sizeof(uint32_t));
    return (p->x && p->vx && p->vy && p->vz && p->z && p->id) ? ORC_OK : ORC_ENOMEM;
}

int orc_create(const orc_config* cfg, orc_sim** out)
{
    if (!cfg || !out) return ORC_EINVAL;
    if (cfg->n_cells < 2 || cfg->length <= 0.0 || cfg->dt <= 0.0 || cfg->eps0 <= 0.0 ||
        cfg->n_species < 1 || cfg->n_species > ORC_MAX_SPECIES ||
        (cfg->bc != ORC_BC_PERIODIC && cfg->bc != ORC_BC_DIRICHLET) ||
        !(cfg->renew_lz >= 0.0 && cfg->renew_lz < 1e300) ||
        cfg->drive < ORC_DRIVE_VOLTAGE || cfg->drive > ORC_DRIVE_CURRENT ||
        (cfg->bc == ORC_BC_PERIODIC && cfg->drive != ORC_DRIVE_VOLTAGE) ||
        (cfg->waveform != ORC_WAVE_SINE && cfg->waveform != ORC_WAVE_TWO_HARMONIC) ||
        !(cfg->cap >= 0.0 && cfg->cap < 1e300) || !(fabs(cfg->j_amp) < 1e300))
        return ORC_EINVAL;
    for (int k = 0; k < cfg->n_species; ++k) {
        if (cfg->sp[k].mass <= 0.0 || cfg->sp[k].capacity < cfg->sp[k].n_init ||
            cfg->sp[k].n_init < 0)
            return ORC_EINVAL;
    }
    orc_sim* s = calloc(1, sizeof(orc_sim));
    if (!s) return ORC_ENOMEM;
    s->c = *cfg;
    s->dx = cfg->length / cfg->n_cells;
    s->nn = cfg->bc == ORC_BC_PERIODIC ? cfg->n_cells : cfg->n_cells + 1;
    int rc = ORC_OK;
    for (int k = 0; k < cfg->n_species; ++k) {
        if (pop_alloc(&s->p[k], cfg->sp[k].capacity) != ORC_OK) rc = ORC_ENOMEM;
        s->sum[k] = calloc((size_t)s->nn, sizeof(double));
        s->dens[k] = calloc((size_t)s->nn, sizeof(double));
        if (!s->sum[k] || !s->dens[k]) rc = ORC_ENOMEM;
    }
    s->rho = calloc((size_t)s->nn, sizeof(double));
    s->phi = calloc((size_t)s->nn, sizeof(double));
    s->ef = calloc((size_t)s->nn, sizeof(double));
    if (!s->rho || !s->phi || !s->ef) rc = ORC_ENOMEM;
    for (int k = 0; k < cfg->n_species; ++k) {
        s->av_dens[k] = calloc((size_t)s->nn, sizeof(double));
        s->av_pw[k] = calloc((size_t)5 * s->nn, sizeof(double));
        s->gprev[k] = calloc((size_t)s->nn, sizeof(double));
        if (!s->av_dens[k] || !s->av_pw[k] || !s->gprev[k]) rc = ORC_ENOMEM;
        s->wedf_emax[k] = k == 0 ? 64.0 : 1024.0;
    }
    s->pw_tmp = calloc((size_t)4 * s->nn, sizeof(double));
    if (!s->pw_tmp) rc = ORC_ENOMEM;
    s->pw_next = UINT64_MAX;
    s->av_phi = calloc((size_t)s->nn, sizeof(double));
    s->av_neps = calloc((size_t)s->nn, sizeof(double));
    if (!s->av_phi || !s->av_neps) rc = ORC_ENOMEM;
    s->eepf_emax = 64.0;
    if (rc != ORC_OK) { orc_free(s); return rc; }
    *out = s;
    return ORC_OK;
}

void orc_free(orc_sim* s)
{
    if (!s) return;
    for (int k = 0; k < ORC_MAX_SPECIES; ++k) {
        free(s->p[k].x); free(s->p[k].vx); free(s->p[k].vy); free(s->p[k].vz); free(s->p[k].id);
        free(s->p[k].z);
        free(s->sum[k]); free(s->dens[k]); free(s->av_dens[k]);
        free(s->av_pw[k]); free(s->gprev[k]);
        free(s->births[k].b);
        for (int j = 0; j < ORC_MAX_CHAN; ++j) { free(s->ch[k][j].e); free(s->ch[k][j].s); }
        free(s->spare[k].x); free(s->spare[k].vx); free(s->spare[k].vy); free(s->spare[k].vz);
        free(s->spare[k].z); free(s->spare[k].id);
    }
    for (int64_t r = 0; r < s->nruns; ++r)
        for (int k = 0; k < ORC_MAX_SPECIES; ++k) free(s->runs[r].births[k].b);
    free(s->runs);
    free(s->part);
    free(s->pw_tmp);
    free(s->rho); free(s->phi); free(s->ef); free(s->av_phi); free(s->av_neps);
    free(s);
}

int orc_load_xsec(orc_sim* s, int32_t sp, int32_t kind, double th, int32_t n,
                  const double* e, const double* sig)
{
    if (!s || sp < 0 || sp >= s->c.n_species || n < 2 || !e || !sig) return ORC_EINVAL;
    if (kind < ORC_XS_ELASTIC || kind > ORC_XS_ION_ISO) return ORC_EINVAL;
    if (s->nch[sp] >= ORC_MAX_CHAN) return ORC_EINVAL;
    if (s->c.gas_density <= 0.0 || s->c.gas_mass <= 0.0) return ORC_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!(e[i] > 0.0) || !(sig[i] >= 0.0) || !isfinite(sig[i]) || !isfinite(e[i]))
            return ORC_EINVAL;
        if (i > 0 && !(e[i] > e[i - 1])) return ORC_EINVAL;
    }
    if (s->nch[sp] > 0 && electron_kind(s->ch[sp][0].kind) != electron_kind(kind))
        return ORC_EINVAL;
    if (kind == ORC_XS_IONIZATION && sp != 0) return ORC_EINVAL;
    chan_t* ch = &s->ch[sp][s->nch[sp]];
    ch->e = malloc((size_t)n * sizeof(double));
    ch->s = malloc((size_t)n * sizeof(double));
    if (!ch->e || !ch->s) return ORC_ENOMEM;
    memcpy(ch->e, e, (size_t)n * sizeof(double));
    memcpy(ch->s, sig, (size_t)n * sizeof(double));
    ch->n = n;
    ch->kind = kind;
    ch->th = th;
    s->nch[sp] += 1;
    update_numax(s, sp);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Charge density on the nodes: each particle gives (1-f) to node c and f to
 * node c+1; a node's density is weight x sum / node volume (dx, or dx/2 at a
 * wall node). */
static void deposit(orc_sim* s)
{
    int nn = s->nn;
    for (int i = 0; i < nn; ++i) s->rho[i] = s->c.rho_bg;
    for (int k = 0; k < s->c.n_species; ++k) {
        double* S = s->sum[k];
        for (int i = 0; i < nn; ++i) S[i] = 0.0;
        for (int64_t p = 0; p < s->p[k].n; ++p) {
            int64_t c, c1;
            double f;
            locate(s, s->p[k].x[p], &c, &c1, &f);
            S[c] += 1.0 - f;
            S[c1] += f;
        }
        for (int i = 0; i < nn; ++i) {
            s->dens[k][i] = s->c.sp[k].weight * S[i] / node_volume(s, i);
            s->rho[i] += s->c.sp[k].charge * s->dens[k][i];
        }
    }
}

/* Poisson -(phi[i-1] - 2 phi[i] + phi[i+1]) / dx^2 = rho[i] / eps0.
 * Dirichlet: phi[0] = V(t), phi[N] = 0, Thomas algorithm on the interior.
 * Periodic: the mean charge is removed, the gauge phi[0] = 0 turns the
 * problem into a Dirichlet one on nodes 1..N-1, and phi is then shifted to
 * zero mean.  Field: central differences inside; at a wall node Gauss's law
 * over the half cell, E0 = -(phi1-phi0)/dx - rho0 dx/(2 eps0) and
 * EN = -(phiN-phiN-1)/dx + rhoN dx/(2 eps0). */
static int solve_dirichlet(const orc_sim* s, double left_bc, const double* rho, double* phi, double* ef)
{
    int nn = s->nn;
    double dx = s->dx, e0 = s->c.eps0;
    if (!s->c.field_solve) {
        for (int i = 0; i < nn; ++i) { phi[i] = 0.0; ef[i] = 0.0; }
        return ORC_OK;
    }
    double* g = malloc((size_t)nn * sizeof(double));
    double* cp = malloc((size_t)nn * sizeof(double));
    double* dp = malloc((size_t)nn * sizeof(double));
    if (!g || !cp || !dp) { free(g); free(cp); free(dp); return ORC_ENOMEM; }
    double left, right;
    if (is_periodic(s)) {
        double mean = 0.0;
        for (int i = 0; i < nn; ++i) mean += rho[i];
        mean /= nn;
        for (int i = 0; i < nn; ++i) g[i] = (rho[i] - mean) * dx * dx / e0;
        left = 0.0;
        right = 0.0;
    } else {
        for (int i = 0; i < nn; ++i) g[i] = rho[i] * dx * dx / e0;
        left = left_bc;
        right = 0.0;
    }
    /* interior unknowns 1..m, m = (periodic ? nn-1 : nn-2); boundary values
     * phi[0] = left and phi[m+1] = right. */
    int m = is_periodic(s) ? nn - 1 : nn - 2;
    for (int i = 1; i <= m; ++i) {
        double d = g[i];
        if (i == 1) d += left;
        if (i == m) d += right;
        double b = 2.0;
        if (i == 1) {
            cp[i] = -1.0 / b;
            dp[i] = d / b;
        } else {
            double den = b + cp[i - 1];         /* b - a c'_{i-1}, a = -1 */
            cp[i] = -1.0 / den;
            dp[i] = (d + dp[i - 1]) / den;
        }
    }
    phi[0] = left;
    if (!is_periodic(s)) phi[nn - 1] = right;
    for (int i = m; i >= 1; --i) {
        double nxt = (i == m) ? 0.0 : phi[i + 1];   /* phi[m+1] already moved to the rhs */
        phi[i] = dp[i] - cp[i] * nxt;
    }
    if (is_periodic(s)) {
        double mean = 0.0;
        for (int i = 0; i < nn; ++i) mean += phi[i];
        mean /= nn;
        for (int i = 0; i < nn; ++i) phi[i] -= mean;
        for (int i = 0; i < nn; ++i) {
            int im = (i == 0) ? nn - 1 : i - 1, ip = (i == nn - 1) ? 0 : i + 1;
            ef[i] = (phi[im] - phi[ip]) / (2.0 * dx);
        }
    } else {
        for (int i = 1; i < nn - 1; ++i) ef[i] = (phi[i - 1] - phi[i + 1]) / (2.0 * dx);
        ef[0] = -(phi[1] - phi[0]) / dx - rho[0] * dx / (2.0 * e0);
        ef[nn - 1] = -(phi[nn - 1] - phi[nn - 2]) / dx + rho[nn - 1] * dx / (2.0 * e0);
    }
    free(g); free(cp); free(dp);
    return ORC_OK;
}

/* The field at time t.  Driven by a voltage, phi(0) is the source.  With an
 * external circuit the electrode's potential follows from its conductor's
 * charge q: the solution is linear in phi0, phi = psi + phi0 (1 - x/L) with
 * psi the solution for phi0 = 0, so the field at the electrode's surface is
 * E0 = E0[psi] + phi0 / L and Gauss's law, q = eps0 E0 + C (phi0 - V(t)),
 * gives phi0 = (C V(t) + q - eps0 E0[psi]) / (C + eps0 / L) (C = 0 for a
 * current source, whose V is zero). */
static int solve(const orc_sim* s, double t, const double* rho, double* phi, double* ef)
{
    if (!circuit_mode(s)) return solve_dirichlet(s, voltage(s, t), rho, phi, ef);
    int rc = solve_dirichlet(s, 0.0, rho, phi, ef);
    if (rc) return rc;
    int nn = s->nn;
    double L = s->c.length, e0 = s->c.eps0;
    double C = s->c.drive == ORC_DRIVE_CAPACITOR ? s->c.cap : 0.0;
    double v = s->c.drive == ORC_DRIVE_CAPACITOR ? source(s, t) : 0.0;
    double q = s->qbase + q_source(s, t) + q_collected(s);
    double p0 = (C * v + q - e0 * ef[0]) / (C + e0 / L);
    for (int i = 0; i < nn; ++i) {
        phi[i] += p0 * (1.0 - (double)i / (double)(nn - 1));
        ef[i] += p0 / L;
    }
    phi[nn - 1] = 0.0;
    return ORC_OK;
}

/* The circuit's charge at the first solve: the electrode starts at the
 * source's potential (capacitor uncharged), or at 0 for a current source. */
static int circuit_start(orc_sim* s, double t)
{
    if (!circuit_mode(s) || s->circ_init) return ORC_OK;
    int nn = s->nn;
    double* phi = malloc((size_t)nn * sizeof(double));
    double* ef = malloc((size_t)nn * sizeof(double));
    if (!phi || !ef) { free(phi); free(ef); return ORC_ENOMEM; }
    int rc = solve_dirichlet(s, 0.0, s->rho, phi, ef);
    double v = s->c.drive == ORC_DRIVE_CAPACITOR ? source(s, t) : 0.0;
    double q = s->c.eps0 * v / s->c.length + s->c.eps0 * ef[0];
    s->qbase = q - q_source(s, t) - q_collected(s);
    s->circ_init = 1;
    free(phi); free(ef);
    return rc;
}

static double field_energy(const orc_sim* s)
{
    double fe = 0.0;
    for (int i = 0; i < s->nn; ++i) fe += s->ef[i] * s->ef[i] * node_volume(s, i);
    return 0.5 * s->c.eps0 * fe;
}

int orc_refresh_field(orc_sim* s)
{
    if (!s) return ORC_EINVAL;
    deposit(s);
    int rc = circuit_start(s, (double)s->step * s->c.dt);
    if (rc) return rc;
    rc = solve(s, (double)s->step * s->c.dt, s->rho, s->phi, s->ef);
    s->fe = field_energy(s);
    return rc;
}

int orc_poisson(const orc_sim* s, double t, const double* rho_in, double* phi_out,
                double* e_out)
{
    if (!s) return ORC_EINVAL;
    int nn = s->nn;
    const double* rho = rho_in ? rho_in : s->rho;
    double* phi = malloc((size_t)nn * sizeof(double));
    double* ef = malloc((size_t)nn * sizeof(double));
    if (!phi || !ef) { free(phi); free(ef); return ORC_ENOMEM; }
    int rc = solve(s, t, rho, phi, ef);
    if (phi_out) memcpy(phi_out, phi, (size_t)nn * sizeof(double));
    if (e_out) memcpy(e_out, ef, (size_t)nn * sizeof(double));
    free(phi); free(ef);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Loading: position from one Philox draw (stratified (j+u)L/N or uniform uL),
 * optionally mapped through the inverse CDF of n0 (1 + eps cos kx) by Newton's
 * method; velocity drift + vth x three Box-Muller normals. */
int orc_load(orc_sim* s)
{
    if (!s) return ORC_EINVAL;
    double L = s->c.length;
    for (int k = 0; k < s->c.n_species; ++k) {
        const orc_species* sp = &s->c.sp[k];
        pop_t* p = &s->p[k];
        int64_t n = sp->load == ORC_LOAD_NONE ? 0 : sp->n_init;
        for (int64_t j = 0; j < n; ++j) {
            uint32_t r0[4], r1[4];
            draw(s, (uint32_t)j, 0xFFFFFFFFu, k, 0u, r0);
            draw(s, (uint32_t)j, 0xFFFFFFFFu, k, 1u, r1);
            double u = orc_u01(r0[0]);
            double x0 = sp->load == ORC_LOAD_STRATIFIED ? ((double)j + u) * L / (double)n : u * L;
            double x = x0;
            if (s->c.perturb_eps != 0.0 && s->c.perturb_mode != 0) {
                double kw = TWO_PI * s->c.perturb_mode / L, ep = s->c.perturb_eps;
                for (int it = 0; it < 60; ++it) {
                    double fx = x + ep / kw * sin(kw * x) - x0;
                    double d = fx / (1.0 + ep * cos(kw * x));
                    x -= d;
                    if (fabs(d) <= 1e-15 * L) break;
                }
            }
            if (x < 0.0) x += L;
            if (x >= L) x -= L;
            double g0, g1, g2, g3;
            box_muller(orc_u01(r1[0]), orc_u01(r1[1]), &g0, &g1);
            box_muller(orc_u01(r1[2]), orc_u01(r1[3]), &g2, &g3);
            p->x[j] = x;
            p->z[j] = 0.0;
            p->vx[j] = sp->drift[0] + sp->vth * g0;
            p->vy[j] = sp->drift[1] + sp->vth * g1;
            p->vz[j] = sp->drift[2] + sp->vth * g2;
            p->id[j] = (uint32_t)j;
        }
        p->n = n;
        p->next_id = (uint32_t)n;
    }
    s->step = 0;
    int rc = orc_refresh_field(s);
    if (rc != ORC_OK) return rc;
    /* leapfrog start: v^{-1/2} = Boris(v^0; E^0, B, -dt/2) */
    for (int k = 0; k < s->c.n_species; ++k) {
        pop_t* p = &s->p[k];
        double qm = s->c.sp[k].charge / s->c.sp[k].mass;
        for (int64_t j = 0; j < p->n; ++j) {
            double e[3] = {gather(s, p->x[j]) + s->c.e_ext[0], s->c.e_ext[1], s->c.e_ext[2]};
            double v[3] = {p->vx[j], p->vy[j], p->vz[j]};
            orc_boris(v, e, s->c.b_ext, qm, -0.5 * s->c.dt);
            p->vx[j] = v[0]; p->vy[j] = v[1]; p->vz[j] = v[2];
        }
    }
    return ORC_OK;
}

/* Start from profiles: density and temperature given at m points evenly
 * spread over [0, L], linear in between.  Position x_j solves F(x) = (j + u_j)/n
 * where F is the integral of the density from 0, divided by its total; it is
 * found by bisection on the exact integral of the linear pieces.  Velocity:
 * three Box-Muller normals times sqrt(e T(x_j) / m).  Then the field at the
 * current step and the leapfrog start, as in orc_load. */
static double profile_integral(const double* d, const double* cum, int m, double h, double x)
{
    /* integral of the linear interpolant of d over [0, x]; cum[i] is the
     * integral over [0, i h] */
    int k = (int)floor(x / h);
    if (k > m - 2) k = m - 2;
    if (k < 0) k = 0;
    double t = x - k * h;
    double slope = (d[k + 1] - d[k]) / h;
    return cum[k] + d[k] * t + 0.5 * slope * t * t;
}

int orc_load_profiles(orc_sim* s, int32_t m, const double* dens, const double* temp_ev,
                      const int64_t* n)
{
    if (!s || m < 2 || !dens || !temp_ev || !n) return ORC_EINVAL;
    double L = s->c.length, h = L / (double)(m - 1);
    for (int k = 0; k < s->c.n_species; ++k) {
        const double* d = dens + (size_t)k * m;
        const double* T = temp_ev + (size_t)k * m;
        double total = 0.0;
        for (int i = 0; i < m; ++i) {
            if (!(d[i] >= 0.0) || !isfinite(d[i]) || !(T[i] >= 0.0) || !isfinite(T[i])) return ORC_EINVAL;
            if (i + 1 < m) total += 0.5 * (d[i] + d[i + 1]) * h;
        }
        if (n[k] < 0 || n[k] > s->p[k].cap || (n[k] > 0 && !(total > 0.0))) return ORC_EINVAL;
    }
    for (int k = 0; k < s->c.n_species; ++k) {
        const double* d = dens + (size_t)k * m;
        const double* T = temp_ev + (size_t)k * m;
        pop_t* p = &s->p[k];
        double* cum = malloc((size_t)m * sizeof(double));
        if (!cum) return ORC_ENOMEM;
        cum[0] = 0.0;
        for (int i = 1; i < m; ++i) cum[i] = cum[i - 1] + 0.5 * (d[i - 1] + d[i]) * h;
        double total = cum[m - 1];
        double mass = s->c.sp[k].mass;
        for (int64_t j = 0; j < n[k]; ++j) {
            uint32_t r0[4], r1[4];
            draw(s, (uint32_t)j, 0xFFFFFFFFu, k, 0u, r0);
            draw(s, (uint32_t)j, 0xFFFFFFFFu, k, 1u, r1);
            double y = ((double)j + orc_u01(r0[0])) / (double)n[k] * total;
            double lo = 0.0, hi = L;
            for (int it = 0; it < 64; ++it) {
                double mid = 0.5 * (lo + hi);
                if (profile_integral(d, cum, m, h, mid) <= y) lo = mid; else hi = mid;
            }
            double x = 0.5 * (lo + hi);
            if (x >= L) x = L * (1.0 - 1e-16);
            int c = (int)floor(x / h);
            if (c > m - 2) c = m - 2;
            double f = x / h - c;
            double Tx = T[c] + f * (T[c + 1] - T[c]);
            double vth = sqrt(s->c.e_unit * Tx / mass);
            double g0, g1, g2, g3;
            box_muller(orc_u01(r1[0]), orc_u01(r1[1]), &g0, &g1);
            box_muller(orc_u01(r1[2]), orc_u01(r1[3]), &g2, &g3);
            p->x[j] = x;
            p->z[j] = 0.0;
            p->vx[j] = vth * g0;
            p->vy[j] = vth * g1;
            p->vz[j] = vth * g2;
            p->id[j] = (uint32_t)j;
        }
        free(cum);
        p->n = n[k];
        s->circ_init = 0;
        p->next_id = (uint32_t)n[k];
    }
    int rc = orc_refresh_field(s);
    if (rc != ORC_OK) return rc;
    for (int k = 0; k < s->c.n_species; ++k) {
        pop_t* p = &s->p[k];
        double qm = s->c.sp[k].charge / s->c.sp[k].mass;
        for (int64_t j = 0; j < p->n; ++j) {
            double e[3] = {gather(s, p->x[j]) + s->c.e_ext[0], s->c.e_ext[1], s->c.e_ext[2]};
            double v[3] = {p->vx[j], p->vy[j], p->vz[j]};
            orc_boris(v, e, s->c.b_ext, qm, -0.5 * s->c.dt);
            p->vx[j] = v[0]; p->vy[j] = v[1]; p->vz[j] = v[2];
        }
    }
    return ORC_OK;
}

int orc_set_particles(orc_sim* s, int32_t k, int64_t n, const double* x, const double* vx,
                      const double* vy, const double* vz, const uint32_t* id,
                      uint32_t next_id)
{
    if (!s || k < 0 || k >= s->c.n_species || n < 0 || n > s->p[k].cap) return ORC_EINVAL;
    pop_t* p = &s->p[k];
    for (int64_t j = 0; j < n; ++j) {
        if (!(x[j] >= 0.0 && x[j] < s->c.length)) return ORC_EINVAL;
        if (!isfinite(vx[j]) || !isfinite(vy[j]) || !isfinite(vz[j])) return ORC_ENUMERIC;
    }
    for (int64_t j = 0; j < n; ++j) {
        p->x[j] = x[j]; p->vx[j] = vx[j]; p->vy[j] = vy[j]; p->vz[j] = vz[j];
        p->id[j] = id[j];
        p->z[j] = 0.0;
    }
    p->n = n;
    p->next_id = next_id;
    s->circ_init = 0;   /* new particles: the circuit restarts at the next solve */
    return ORC_OK;
}

/* Axial displacements of species k (renewal, Lafleur's method): replace the
 * first n values (n = the species' count) or read them. */
int orc_set_axial(orc_sim* s, int32_t k, int64_t n, const double* z)
{
    if (!s || k < 0 || k >= s->c.n_species || !z || n != s->p[k].n) return ORC_EINVAL;
    for (int64_t j = 0; j < n; ++j) {
        if (!isfinite(z[j])) return ORC_ENUMERIC;
        s->p[k].z[j] = z[j];
    }
    return ORC_OK;
}

int orc_get_axial(const orc_sim* s, int32_t k, int64_t cap, double* z)
{
    if (!s || k < 0 || k >= s->c.n_species || !z || cap < s->p[k].n) return ORC_EINVAL;
    for (int64_t j = 0; j < s->p[k].n; ++j) z[j] = s->p[k].z[j];
    return ORC_OK;
}

int orc_get_particles(const orc_sim* s, int32_t k, int64_t cap, double* x, double* vx,
                      double* vy, double* vz, uint32_t* id, int64_t* n, uint32_t* next_id)
{
    if (!s || k < 0 || k >= s->c.n_species) return ORC_EINVAL;
    const pop_t* p = &s->p[k];
    if (n) *n = p->n;
    if (next_id) *next_id = p->next_id;
    if (cap < p->n) return x ? ORC_EINVAL : ORC_OK;
    for (int64_t j = 0; j < p->n; ++j) {
        if (x) x[j] = p->x[j];
        if (vx) vx[j] = p->vx[j];
        if (vy) vy[j] = p->vy[j];
        if (vz) vz[j] = p->vz[j];
        if (id) id[j] = p->id[j];
    }
    return ORC_OK;
}

int orc_set_step(orc_sim* s, uint64_t step) { if (!s) return ORC_EINVAL; s->step = step; return ORC_OK; }
uint64_t orc_get_step(const orc_sim* s) { return s ? s->step : 0; }

/* ------------------------------------------------------------------------ */
static int push_birth(blist_t* l, double x, double vx, double vy, double vz)
{
    if (l->n == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 1024;
        birth_t* nb = realloc(l->b, (size_t)nc * sizeof(birth_t));
        if (!nb) return ORC_ENOMEM;
        l->b = nb;
        l->cap = nc;
    }
    l->b[l->n].x = x; l->b[l->n].vx = vx; l->b[l->n].vy = vy; l->b[l->n].vz = vz;
    l->n += 1;
    return ORC_OK;
}

/* Null-collision Monte Carlo for one particle of species k at position x with
 * velocity v (modified in place).  Draw 0 decides candidacy by the integer
 * test x0 < T32, picks the channel with u1 nu_max against the running sum of
 * nu_k = n_g sigma_k v, and gives the scattering angles cos(chi) = 1 - 2 u2,
 * phi = 2 pi u3. */
static int collide(const orc_sim* s, sink_t* o, int k, uint32_t id, double x, double v[3])
{
    int nch = s->nch[k];
    uint32_t r[4];
    draw(s, id, (uint32_t)s->step, k, 0u, r);
    if (r[0] >= s->t32[k]) return ORC_OK;
    o->cnt.candidates[k] += 1;
    double m = s->c.sp[k].mass, M = s->c.gas_mass, ng = s->c.gas_density;
    double eu = s->c.e_unit;
    int ion = !electron_kind(s->ch[k][0].kind);
    double nu[ORC_MAX_CHAN];
    double vn[3] = {0.0, 0.0, 0.0};
    double speed, eps;
    if (!ion) {
        double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        speed = sqrt(v2);
        eps = 0.5 * m * v2 / eu;
    } else {
        uint32_t r3[4];
        draw(s, id, (uint32_t)s->step, k, 3u, r3);
        double g0, g1, g2, g3, vt = sqrt(K_B * s->c.gas_temp / M);
        box_muller(orc_u01(r3[0]), orc_u01(r3[1]), &g0, &g1);
        box_muller(orc_u01(r3[2]), orc_u01(r3[3]), &g2, &g3);
        vn[0] = vt * g0; vn[1] = vt * g1; vn[2] = vt * g2;
        double gx = v[0] - vn[0], gy = v[1] - vn[1], gz = v[2] - vn[2];
        double g2s = gx * gx + gy * gy + gz * gz;
        speed = sqrt(g2s);
        eps = 0.5 * m * g2s / eu;
    }
    double total = 0.0;
    for (int c = 0; c < nch; ++c) {
        nu[c] = ng * sigma_at(&s->ch[k][c], eps) * speed;
        total += nu[c];
    }
    if (total > s->numax[k]) o->cnt.violations[k] += 1;
    double u1 = orc_u01(r[1]);
    double target = u1 * s->numax[k];
    double cum = 0.0;
    int chosen = -1;
    for (int c = 0; c < nch; ++c) {
        cum += nu[c];
        if (target < cum) { chosen = c; break; }
    }
    if (chosen < 0) { o->cnt.nulls[k] += 1; return ORC_OK; }
    o->cnt.coll[k][chosen] += 1;
    double cos_chi = 1.0 - 2.0 * orc_u01(r[2]);
    double phi = TWO_PI * orc_u01(r[3]);
    const chan_t* ch = &s->ch[k][chosen];
    if (!ion) {
        double d[3] = {v[0] / speed, v[1] / speed, v[2] / speed};
        double nd[3];
        orc_rotate(d, cos_chi, phi, nd);
        double eps_new;
        if (ch->kind == ORC_XS_ELASTIC) {
            eps_new = eps * (1.0 - 2.0 * m / M * (1.0 - cos_chi));
        } else if (ch->kind == ORC_XS_EXCITATION) {
            eps_new = eps - ch->th;
        } else {  /* ionization: uniform split of eps - threshold */
            uint32_t r1[4], r2[4];
            draw(s, id, (uint32_t)s->step, k, 1u, r1);
            draw(s, id, (uint32_t)s->step, k, 2u, r2);
            double avail = eps - ch->th;
            double eps_ej = orc_u01(r1[0]) * avail;
            eps_new = avail - eps_ej;
            double ed[3];
            orc_rotate(d, 1.0 - 2.0 * orc_u01(r1[1]), TWO_PI * orc_u01(r1[2]), ed);
            double vej = sqrt(2.0 * eps_ej * eu / m);
            int rc = push_birth(&o->births[0], x, vej * ed[0], vej * ed[1], vej * ed[2]);
            if (rc) return rc;
            double g0, g1, g2, g3, vt = sqrt(K_B * s->c.gas_temp / M);
            box_muller(orc_u01(r2[0]), orc_u01(r2[1]), &g0, &g1);
            box_muller(orc_u01(r2[2]), orc_u01(r2[3]), &g2, &g3);
            if (s->c.n_species > 1) {   /* with electrons only (a swarm) the ion is not followed */
                rc = push_birth(&o->births[1], x, vt * g0, vt * g1, vt * g2);
                if (rc) return rc;
            }
        }
        if (eps_new < 0.0) eps_new = 0.0;
        double vs = sqrt(2.0 * eps_new * eu / m);
        v[0] = vs * nd[0]; v[1] = vs * nd[1]; v[2] = vs * nd[2];
    } else {
        if (ch->kind == ORC_XS_ION_CX) {            /* charge exchange: ion takes vn */
            v[0] = vn[0]; v[1] = vn[1]; v[2] = vn[2];
        } else {                                     /* isotropic in the centre of mass */
            double mt = m + M;
            double vc[3] = {(m * v[0] + M * vn[0]) / mt, (m * v[1] + M * vn[1]) / mt,
                            (m * v[2] + M * vn[2]) / mt};
            double st = sqrt(fmax(0.0, 1.0 - cos_chi * cos_chi));
            double gd[3] = {cos_chi, st * cos(phi), st * sin(phi)};
            double f = M / mt * speed;
            v[0] = vc[0] + f * gd[0]; v[1] = vc[1] + f * gd[1]; v[2] = vc[2] + f * gd[2];
        }
    }
    return ORC_OK;
}

/* Secondary electron from an ion absorbed at wall w (0: x = 0, 1: x = L):
 * emitted with probability gamma; normal speed from the flux-weighted
 * half-Maxwellian v_see sqrt(-2 ln u), tangential components Maxwellian,
 * advanced into the gap by u v_n dt. */
static int emit_secondary(const orc_sim* s, sink_t* o, int k, uint32_t id, int wall)
{
    uint32_t r4[4], r5[4];
    draw(s, id, (uint32_t)s->step, k, 4u, r4);
    if (!(orc_u01(r4[0]) < s->c.see_gamma)) return ORC_OK;
    draw(s, id, (uint32_t)s->step, k, 5u, r5);
    double vsee = sqrt(s->c.see_temp * s->c.e_unit / s->c.sp[0].mass);
    double vn = vsee * sqrt(-2.0 * log(orc_u01(r4[1])));
    double adv = orc_u01(r4[2]) * vn * s->c.dt;
    double g0, g1;
    box_muller(orc_u01(r5[0]), orc_u01(r5[1]), &g0, &g1);
    if (adv >= s->c.length) { o->cnt.dropped += 1; return ORC_OK; }
    double x = wall == 0 ? adv : s->c.length - adv;
    double vx = wall == 0 ? vn : -vn;
    if (!(x >= 0.0 && x < s->c.length)) { o->cnt.dropped += 1; return ORC_OK; }
    o->cnt.see_emitted[wall] += 1;
    return push_birth(&o->births[0], x, vx, vsee * g0, vsee * g1);
}

/* Energy histograms: bin floor(eps / width) with width = emax / ORC_EEPF_BINS;
 * energies at or above emax are not counted. */
static void tally(int64_t* h, double eps, double emax)
{
    double b = floor(eps * (double)ORC_EEPF_BINS / emax);
    if (b >= 0.0 && b < (double)ORC_EEPF_BINS) h[(int)b] += 1;
}

/* Cells whose electrons make up the bulk energy distribution: the whole
 * domain when periodic, else the middle tenth of the gap, cells
 * floor(0.45 N) .. max(that + 1, ceil(0.55 N)) - 1. */
static void bulk_cells(const orc_sim* s, int64_t* lo, int64_t* hi)
{
    int64_t nc = s->c.n_cells;
    if (is_periodic(s)) { *lo = 0; *hi = nc; return; }
    *lo = (int64_t)floor(0.45 * (double)nc);
    *hi = (int64_t)ceil(0.55 * (double)nc);
    if (*hi < *lo + 1) *hi = *lo + 1;
}

/* One sample of the time-accumulated diagnostics, taken on the state at the
 * end of a step (positions x^{n+1}, velocities v^{n+1/2} after collisions,
 * births included): the densities and the potential at the nodes, the
 * electron energy density sum_p S_i(x_p) eps_p w / V_i (its ratio to the
 * electron density is the mean energy), and the bulk electron energy
 * histogram. */
static void sample_diagnostics(orc_sim* s)
{
    int nn = s->nn;
    for (int k = 0; k < s->c.n_species; ++k)
        for (int i = 0; i < nn; ++i) s->av_dens[k][i] += s->dens[k][i];
    for (int i = 0; i < nn; ++i) s->av_phi[i] += s->phi[i];
    const pop_t* e = &s->p[0];
    double* ne = s->sum[0];             /* reused as the energy sums of this sample */
    for (int i = 0; i < nn; ++i) ne[i] = 0.0;
    int64_t lo, hi;
    bulk_cells(s, &lo, &hi);
    for (int64_t p = 0; p < e->n; ++p) {
        double v2 = e->vx[p] * e->vx[p] + e->vy[p] * e->vy[p] + e->vz[p] * e->vz[p];
        double eps = 0.5 * s->c.sp[0].mass * v2 / s->c.e_unit;
        int64_t c, c1;
        double f;
        locate(s, e->x[p], &c, &c1, &f);
        ne[c] += (1.0 - f) * eps;
        ne[c1] += f * eps;
        if (c >= lo && c < hi) tally(s->eepf[0], eps, s->eepf_emax);
    }
    for (int i = 0; i < nn; ++i) {
        s->av_neps[i] += s->c.sp[0].weight * ne[i] / node_volume(s, i);
        ne[i] = 0.0;
    }
    s->av_samples += 1.0;
}

/* The power the field gives each species, and its decomposition (the paper
 * names the power terms without formulas; the reading is the momentum
 * balance of the species, m dGamma/dt + d(m n <vx^2>)/dx = q n E + R, times
 * its mean velocity u = Gamma / n):
 *   q Gamma E = u (m dGamma/dt + d(m Gamma^2/n)/dx)   inertia
 *             + u dp/dx,  p = m (n <vx^2> - Gamma^2/n)  pressure
 *             + ohmic (the rest: -u R, the momentum lost in collisions).
 * Gamma = w sum_p S_i(x_p) vx_p / V_i and n <vx^2> likewise, at the state
 * the step ends with; dGamma/dt by the flux of the previous step when that
 * step was sampled, else 0; gradients central inside, one-sided at a wall
 * node; E is the mesh field plus the imposed one.  Accumulated per node:
 * Gamma, n <vx^2>, q Gamma E, inertia, pressure.  flux and mom hold species
 * k's Gamma and n <vx^2>. */
static void sample_power(orc_sim* s, int k, const double* flux, const double* mom, int prev)
{
    int nn = s->nn, periodic = is_periodic(s);
    double m = s->c.sp[k].mass, dt = s->c.dt;
    double* kt = s->pw_tmp + 2 * nn;
    double* pt = s->pw_tmp + 3 * nn;
    for (int i = 0; i < nn; ++i) {
        double n = s->dens[k][i];
        kt[i] = n > 0.0 ? m * flux[i] * flux[i] / n : 0.0;
        pt[i] = m * mom[i] - kt[i];
    }
    double* av = s->av_pw[k];
    for (int i = 0; i < nn; ++i) {
        int il, ir;
        double h;
        if (periodic) {
            il = i == 0 ? nn - 1 : i - 1;
            ir = i == nn - 1 ? 0 : i + 1;
            h = 2.0 * s->dx;
        } else {
            il = i > 0 ? i - 1 : i;
            ir = i < nn - 1 ? i + 1 : i;
            h = (double)(ir - il) * s->dx;
        }
        double n = s->dens[k][i];
        double u = n > 0.0 ? flux[i] / n : 0.0;
        double dgdt = prev ? (flux[i] - s->gprev[k][i]) / dt : 0.0;
        av[i] += flux[i];
        av[nn + i] += mom[i];
        av[2 * nn + i] += s->c.sp[k].charge * flux[i] * (s->ef[i] + s->c.e_ext[0]);
        av[3 * nn + i] += u * (m * dgdt + (kt[ir] - kt[il]) / h);
        av[4 * nn + i] += u * (pt[ir] - pt[il]) / h;
        s->gprev[k][i] = flux[i];
    }
}

static int grow_part(orc_sim* s, int64_t n);

/* The sequential sample of every species' power terms. */
static void sample_power_all(orc_sim* s)
{
    int prev = s->pw_next == s->step;
    double* flux = s->pw_tmp;
    double* mom = s->pw_tmp + s->nn;
    for (int k = 0; k < s->c.n_species; ++k) {
        orc_get_moments(s, k, flux, mom);
        sample_power(s, k, flux, mom, prev);
    }
    s->pw_next = s->step + 1;
}

/* The same with the moments summed per chunk of particles and over chunks
 * in order (the parallel step). */
static void sample_power_chunks(orc_sim* s)
{
    int nn = s->nn, prev = s->pw_next == s->step;
    double* flux = s->pw_tmp;
    double* mom = s->pw_tmp + nn;
    for (int k = 0; k < s->c.n_species; ++k) {
        const pop_t* p = &s->p[k];
        int64_t nchunk = (p->n + ORC_CHUNK - 1) / ORC_CHUNK;
        if (grow_part(s, nchunk * 2 * nn) != ORC_OK) {
            orc_get_moments(s, k, flux, mom);
            sample_power(s, k, flux, mom, prev);
            continue;
        }
        double* part = s->part;
        #pragma omp parallel for schedule(static) num_threads(s->threads)
        for (int64_t ck = 0; ck < nchunk; ++ck) {
            double* F = part + ck * 2 * nn;
            double* M = F + nn;
            for (int i = 0; i < 2 * nn; ++i) F[i] = 0.0;
            int64_t j1 = (ck + 1) * ORC_CHUNK < p->n ? (ck + 1) * ORC_CHUNK : p->n;
            for (int64_t j = ck * ORC_CHUNK; j < j1; ++j) {
                int64_t c, c1;
                double f, vx = p->vx[j];
                locate(s, p->x[j], &c, &c1, &f);
                F[c] += (1.0 - f) * vx;
                F[c1] += f * vx;
                M[c] += (1.0 - f) * vx * vx;
                M[c1] += f * vx * vx;
            }
        }
        for (int i = 0; i < nn; ++i) {
            double a = 0.0, b = 0.0;
            for (int64_t ck = 0; ck < nchunk; ++ck) {
                a += part[ck * 2 * nn + i];
                b += part[ck * 2 * nn + nn + i];
            }
            flux[i] = a * s->c.sp[k].weight / node_volume(s, i);
            mom[i] = b * s->c.sp[k].weight / node_volume(s, i);
        }
        sample_power(s, k, flux, mom, prev);
    }
    s->pw_next = s->step + 1;
}

int orc_get_power(const orc_sim* s, int32_t k, double* out)
{
    if (!s || k < 0 || k >= s->c.n_species || !out) return ORC_EINVAL;
    for (int i = 0; i < 5 * s->nn; ++i) out[i] = s->av_samples > 0.0 ? s->av_pw[k][i] / s->av_samples : 0.0;
    return ORC_OK;
}

/* Axial renewal (Lafleur, Baalrud and Chabert): each particle carries the
 * virtual displacement z along the imposed field's axis (the third velocity
 * component) since its injection, advanced with the new velocity; once
 * |z| >= L_z the particle is re-injected at the same x with a fresh velocity
 * from the species' initial distribution (Maxwellian of scale vth plus the
 * drift), drawn with call 6, and z = 0. */
static void renew(const orc_sim* s, sink_t* o, int k, uint32_t id, double v[3], double* z)
{
    *z += v[2] * s->c.dt;
    if (fabs(*z) < s->c.renew_lz) return;
    uint32_t r[4];
    draw(s, id, (uint32_t)s->step, k, 6u, r);
    double g0, g1, g2, g3;
    box_muller(orc_u01(r[0]), orc_u01(r[1]), &g0, &g1);
    box_muller(orc_u01(r[2]), orc_u01(r[3]), &g2, &g3);
    const orc_species* sp = &s->c.sp[k];
    v[0] = sp->drift[0] + sp->vth * g0;
    v[1] = sp->drift[1] + sp->vth * g1;
    v[2] = sp->drift[2] + sp->vth * g2;
    *z = 0.0;
    o->cnt.renewed[k] += 1;
}

/* One particle's step: gather E at x^n, Boris to v^{n+1/2}, move to x^{n+1},
 * wrap or absorb (with secondary emission), renew, collide.  Returns 1 when
 * the particle stays (x, v, z updated), 0 when it is absorbed; side effects
 * go to the run's sink o. */
static int step_particle(const orc_sim* s, sink_t* o, int k, uint32_t id, double* xp, double v[3], double* z)
{
    double L = s->c.length, dt = s->c.dt;
    double qm = s->c.sp[k].charge / s->c.sp[k].mass;
    double half_mw = 0.5 * s->c.sp[k].mass * s->c.sp[k].weight;
    double x = *xp;
    double vold2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double e[3] = {gather(s, x) + s->c.e_ext[0], s->c.e_ext[1], s->c.e_ext[2]};
    orc_boris(v, e, s->c.b_ext, qm, dt);
    double vnew2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    o->ke += half_mw * 0.5 * (vold2 + vnew2);
    x += v[0] * dt;
    if (is_periodic(s)) {
        if (x < 0.0) x += L;
        if (x >= L) x -= L;
    } else if (x < 0.0 || x >= L) {
        int wall = x < 0.0 ? 0 : 1;
        o->cnt.absorbed[k][wall] += 1;
        o->cnt.wall_energy[k][wall] += half_mw * vnew2;
        if (s->diag) {
            double eps = 0.5 * s->c.sp[k].mass * vnew2 / s->c.e_unit;
            tally(o->wedf[wall], eps, s->wedf_emax[k]);
            if (k == 0) tally(o->eepf_wall, eps, s->eepf_emax);
        }
        if (k > 0 && s->c.sp[k].charge > 0.0 && s->c.see_gamma > 0.0) {
            int rc = emit_secondary(s, o, k, id, wall);
            if (rc && !o->rc) o->rc = rc;
        }
        return 0;
    }
    if (s->c.renew_lz > 0.0) renew(s, o, k, id, v, z);
    if (s->nch[k] > 0) {
        int rc = collide(s, o, k, id, x, v);
        if (rc && !o->rc) o->rc = rc;
    }
    *xp = x;
    return 1;
}

static void run_reset(const orc_sim* s, sink_t* o)
{
    memset(&o->cnt, 0, sizeof(o->cnt));
    for (int k = 0; k < ORC_MAX_SPECIES; ++k) o->births[k].n = 0;
    o->ke = 0.0;
    if (s->diag) {
        memset(o->eepf_wall, 0, sizeof(o->eepf_wall));
        memset(o->wedf, 0, sizeof(o->wedf));
    }
    o->keep = 0;
    o->rc = ORC_OK;
}

/* Add a run of species k to the step's totals: counters, kinetic energy,
 * histograms, and its births after the ones already made this step. */
static int run_merge(orc_sim* s, int k, const sink_t* o)
{
    orc_counters* c = &s->cnt;
    for (int q = 0; q < ORC_MAX_SPECIES; ++q) {
        for (int w = 0; w < 2; ++w) {
            c->absorbed[q][w] += o->cnt.absorbed[q][w];
            c->wall_energy[q][w] += o->cnt.wall_energy[q][w];
        }
        c->candidates[q] += o->cnt.candidates[q];
        c->nulls[q] += o->cnt.nulls[q];
        for (int j = 0; j < ORC_MAX_CHAN; ++j) c->coll[q][j] += o->cnt.coll[q][j];
        c->violations[q] += o->cnt.violations[q];
        c->renewed[q] += o->cnt.renewed[q];
    }
    for (int w = 0; w < 2; ++w) c->see_emitted[w] += o->cnt.see_emitted[w];
    c->dropped += o->cnt.dropped;
    s->ke[k] += o->ke;
    if (s->diag) {
        for (int i = 0; i < ORC_EEPF_BINS; ++i) {
            s->eepf[1][i] += o->eepf_wall[i];
            s->wedf[k][0][i] += o->wedf[0][i];
            s->wedf[k][1][i] += o->wedf[1][i];
        }
    }
    for (int q = 0; q < ORC_MAX_SPECIES; ++q)
        for (int64_t b = 0; b < o->births[q].n; ++b) {
            const birth_t* bb = &o->births[q].b[b];
            int rc = push_birth(&s->births[q], bb->x, bb->vx, bb->vy, bb->vz);
            if (rc) return rc;
        }
    return o->rc;
}

/* The step's births appended after the survivors, in the order they were
 * made, with ids from the species counter. */
static int append_births(orc_sim* s)
{
    int rc = ORC_OK;
    for (int k = 0; k < s->c.n_species; ++k) {
        pop_t* p = &s->p[k];
        for (int64_t b = 0; b < s->births[k].n; ++b) {
            if (p->n >= p->cap) { s->cnt.dropped += s->births[k].n - b; rc = ORC_ECAPACITY; break; }
            const birth_t* bb = &s->births[k].b[b];
            p->x[p->n] = bb->x; p->vx[p->n] = bb->vx; p->vy[p->n] = bb->vy; p->vz[p->n] = bb->vz;
            p->z[p->n] = 0.0;
            p->id[p->n] = p->next_id++;
            p->n += 1;
        }
    }
    return rc;
}

static int grow_runs(orc_sim* s, int64_t n)
{
    if (n <= s->nruns) return ORC_OK;
    sink_t* r = realloc(s->runs, (size_t)n * sizeof(sink_t));
    if (!r) return ORC_ENOMEM;
    memset(r + s->nruns, 0, (size_t)(n - s->nruns) * sizeof(sink_t));
    s->runs = r;
    s->nruns = n;
    return ORC_OK;
}

static void deposit_chunks(orc_sim* s);
static void sample_diagnostics_chunks(orc_sim* s);

/* One leapfrog step: for each species in order, each particle in index order
 * (step_particle).  Survivors keep their order; births follow, in the order
 * they were made, with ids from the species counter.  Then the deposit, and
 * the field at t^{n+1}.
 *
 * Sequential (threads == 0): one run per species, plain loops.  Parallel
 * (threads > 0, OpenMP): the particles of a species in chunks of ORC_CHUNK,
 * each its own run, survivors written to a second population and moved back
 * in chunk order, runs merged in chunk order, the deposit and the sampled
 * diagnostics summed per chunk and then over chunks in order; the result is
 * the same for every thread count, and differs from the sequential one only
 * in the rounding of those sums. */
static int one_step(orc_sim* s)
{
    double dt = s->c.dt;
    for (int k = 0; k < s->c.n_species; ++k) s->births[k].n = 0;
    int rc = grow_runs(s, 1);
    if (rc) return rc;
    for (int k = 0; k < s->c.n_species; ++k) {
        pop_t* p = &s->p[k];
        s->ke[k] = 0.0;
        if (s->threads <= 0) {
            sink_t* o = &s->runs[0];
            run_reset(s, o);
            int64_t keep = 0;
            for (int64_t j = 0; j < p->n; ++j) {
                double x = p->x[j];
                double v[3] = {p->vx[j], p->vy[j], p->vz[j]};
                double z = p->z[j];
                if (!step_particle(s, o, k, p->id[j], &x, v, &z)) continue;
                p->x[keep] = x;
                p->vx[keep] = v[0]; p->vy[keep] = v[1]; p->vz[keep] = v[2];
                p->z[keep] = z;
                p->id[keep] = p->id[j];
                keep += 1;
            }
            p->n = keep;
            rc = run_merge(s, k, o);
            if (rc) return rc;
            continue;
        }
        int64_t nchunk = (p->n + ORC_CHUNK - 1) / ORC_CHUNK;
        rc = grow_runs(s, nchunk);
        if (rc) return rc;
        pop_t* q = &s->spare[k];
        if (q->cap < p->cap) {
            free(q->x); free(q->vx); free(q->vy); free(q->vz); free(q->z); free(q->id);
            rc = pop_alloc(q, p->cap);
            if (rc) return rc;
        }
        #pragma omp parallel for schedule(dynamic, 1) num_threads(s->threads)
        for (int64_t ck = 0; ck < nchunk; ++ck) {
            sink_t* o = &s->runs[ck];
            run_reset(s, o);
            int64_t j0 = ck * ORC_CHUNK, j1 = j0 + ORC_CHUNK < p->n ? j0 + ORC_CHUNK : p->n;
            for (int64_t j = j0; j < j1; ++j) {
                double x = p->x[j];
                double v[3] = {p->vx[j], p->vy[j], p->vz[j]};
                double z = p->z[j];
                if (!step_particle(s, o, k, p->id[j], &x, v, &z)) continue;
                int64_t d = j0 + o->keep++;
                q->x[d] = x;
                q->vx[d] = v[0]; q->vy[d] = v[1]; q->vz[d] = v[2];
                q->z[d] = z;
                q->id[d] = p->id[j];
            }
        }
        /* survivors back in chunk order */
        int64_t keep = 0;
        for (int64_t ck = 0; ck < nchunk; ++ck) {
            int64_t kc = s->runs[ck].keep;
            s->runs[ck].keep = keep;         /* now: the chunk's first survivor slot */
            keep += kc;
        }
        #pragma omp parallel for schedule(static) num_threads(s->threads)
        for (int64_t ck = 0; ck < nchunk; ++ck) {
            int64_t d = s->runs[ck].keep, src = ck * ORC_CHUNK;
            int64_t kc = (ck + 1 < nchunk ? s->runs[ck + 1].keep : keep) - d;
            memcpy(p->x + d, q->x + src, (size_t)kc * sizeof(double));
            memcpy(p->vx + d, q->vx + src, (size_t)kc * sizeof(double));
            memcpy(p->vy + d, q->vy + src, (size_t)kc * sizeof(double));
            memcpy(p->vz + d, q->vz + src, (size_t)kc * sizeof(double));
            memcpy(p->z + d, q->z + src, (size_t)kc * sizeof(double));
            memcpy(p->id + d, q->id + src, (size_t)kc * sizeof(uint32_t));
        }
        p->n = keep;
        for (int64_t ck = 0; ck < nchunk; ++ck) {
            rc = run_merge(s, k, &s->runs[ck]);
            if (rc) return rc;
        }
    }
    rc = append_births(s);
    s->step += 1;
    if (s->threads <= 0) deposit(s); else deposit_chunks(s);
    int rs = circuit_start(s, (double)s->step * dt);
    if (rs == ORC_OK) rs = solve(s, (double)s->step * dt, s->rho, s->phi, s->ef);
    s->fe = field_energy(s);
    if (s->diag) {
        if (s->threads <= 0) {
            sample_power_all(s);
            sample_diagnostics(s);
        } else {
            sample_power_chunks(s);
            sample_diagnostics_chunks(s);
        }
    }
    return rc != ORC_OK ? rc : rs;
}

/* The deposit of the parallel step: per chunk of particles, the sums of the
 * linear weights at the nodes; then, node by node, the sum over chunks in
 * chunk order. */
static int grow_part(orc_sim* s, int64_t n)
{
    if (n <= s->npart) return ORC_OK;
    double* p = realloc(s->part, (size_t)n * sizeof(double));
    if (!p) return ORC_ENOMEM;
    s->part = p;
    s->npart = n;
    return ORC_OK;
}

static void deposit_chunks(orc_sim* s)
{
    int nn = s->nn;
    for (int i = 0; i < nn; ++i) s->rho[i] = s->c.rho_bg;
    for (int k = 0; k < s->c.n_species; ++k) {
        const pop_t* p = &s->p[k];
        double* S = s->sum[k];
        int64_t nchunk = (p->n + ORC_CHUNK - 1) / ORC_CHUNK;
        if (grow_part(s, nchunk * nn) != ORC_OK) { deposit(s); return; }
        double* part = s->part;
        #pragma omp parallel for schedule(static) num_threads(s->threads)
        for (int64_t ck = 0; ck < nchunk; ++ck) {
            double* P = part + ck * nn;
            for (int i = 0; i < nn; ++i) P[i] = 0.0;
            int64_t j1 = (ck + 1) * ORC_CHUNK < p->n ? (ck + 1) * ORC_CHUNK : p->n;
            for (int64_t j = ck * ORC_CHUNK; j < j1; ++j) {
                int64_t c, c1;
                double f;
                locate(s, p->x[j], &c, &c1, &f);
                P[c] += 1.0 - f;
                P[c1] += f;
            }
        }
        #pragma omp parallel for schedule(static) num_threads(s->threads)
        for (int i = 0; i < nn; ++i) {
            double t = 0.0;
            for (int64_t ck = 0; ck < nchunk; ++ck) t += part[ck * nn + i];
            S[i] = t;
        }
        for (int i = 0; i < nn; ++i) {
            s->dens[k][i] = s->c.sp[k].weight * S[i] / node_volume(s, i);
            s->rho[i] += s->c.sp[k].charge * s->dens[k][i];
        }
    }
}

/* The sampled diagnostics of the parallel step: the electron energy at the
 * nodes summed per chunk and over chunks in order, the bulk histogram per
 * chunk (integers). */
static void sample_diagnostics_chunks(orc_sim* s)
{
    int nn = s->nn;
    for (int k = 0; k < s->c.n_species; ++k)
        for (int i = 0; i < nn; ++i) s->av_dens[k][i] += s->dens[k][i];
    for (int i = 0; i < nn; ++i) s->av_phi[i] += s->phi[i];
    const pop_t* e = &s->p[0];
    int64_t nchunk = (e->n + ORC_CHUNK - 1) / ORC_CHUNK;
    if (grow_part(s, nchunk * nn) != ORC_OK || grow_runs(s, nchunk) != ORC_OK) {
        /* no room for the chunk sums: undo this sample's fields, take it sequentially */
        for (int k = 0; k < s->c.n_species; ++k)
            for (int i = 0; i < nn; ++i) s->av_dens[k][i] -= s->dens[k][i];
        for (int i = 0; i < nn; ++i) s->av_phi[i] -= s->phi[i];
        sample_diagnostics(s);
        return;
    }
    double* part = s->part;
    int64_t lo, hi;
    bulk_cells(s, &lo, &hi);
    #pragma omp parallel for schedule(static) num_threads(s->threads)
    for (int64_t ck = 0; ck < nchunk; ++ck) {
        double* P = part + ck * nn;
        int64_t* H = s->runs[ck].eepf_wall;          /* reused as this chunk's bulk histogram */
        for (int i = 0; i < nn; ++i) P[i] = 0.0;
        for (int i = 0; i < ORC_EEPF_BINS; ++i) H[i] = 0;
        int64_t j1 = (ck + 1) * ORC_CHUNK < e->n ? (ck + 1) * ORC_CHUNK : e->n;
        for (int64_t p = ck * ORC_CHUNK; p < j1; ++p) {
            double v2 = e->vx[p] * e->vx[p] + e->vy[p] * e->vy[p] + e->vz[p] * e->vz[p];
            double eps = 0.5 * s->c.sp[0].mass * v2 / s->c.e_unit;
            int64_t c, c1;
            double f;
            locate(s, e->x[p], &c, &c1, &f);
            P[c] += (1.0 - f) * eps;
            P[c1] += f * eps;
            if (c >= lo && c < hi) tally(H, eps, s->eepf_emax);
        }
    }
    for (int i = 0; i < nn; ++i) {
        double t = 0.0;
        for (int64_t ck = 0; ck < nchunk; ++ck) t += part[ck * nn + i];
        s->av_neps[i] += s->c.sp[0].weight * t / node_volume(s, i);
    }
    for (int64_t ck = 0; ck < nchunk; ++ck)
        for (int i = 0; i < ORC_EEPF_BINS; ++i) s->eepf[0][i] += s->runs[ck].eepf_wall[i];
    s->av_samples += 1.0;
}

int orc_set_threads(orc_sim* s, int32_t threads)
{
    if (!s || threads < 0) return ORC_EINVAL;
    s->threads = threads;
    return ORC_OK;
}

int orc_step(orc_sim* s, int32_t n)
{
    if (!s || n < 0) return ORC_EINVAL;
    for (int32_t i = 0; i < n; ++i) {
        int rc = one_step(s);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
int orc_n_nodes(const orc_sim* s) { return s ? s->nn : 0; }

int orc_get_field(const orc_sim* s, double* rho, double* phi, double* efield)
{
    if (!s) return ORC_EINVAL;
    size_t b = (size_t)s->nn * sizeof(double);
    if (rho) memcpy(rho, s->rho, b);
    if (phi) memcpy(phi, s->phi, b);
    if (efield) memcpy(efield, s->ef, b);
    return ORC_OK;
}

int orc_get_density(const orc_sim* s, int32_t k, double* dens)
{
    if (!s || k < 0 || k >= s->c.n_species || !dens) return ORC_EINVAL;
    memcpy(dens, s->dens[k], (size_t)s->nn * sizeof(double));
    return ORC_OK;
}

/* Velocity moments of species k at the nodes, with the weights of the charge
 * deposit: flux[i] = w sum_p S_i(x_p) vx_p / V_i and mom[i] = w sum_p S_i(x_p)
 * vx_p^2 / V_i (S_i the linear weight of node i, V_i its volume); with the
 * field E[i] at the same nodes, q flux[i] E[i] is the power density the field
 * gives the species. */
int orc_get_moments(const orc_sim* s, int32_t k, double* flux, double* mom)
{
    if (!s || k < 0 || k >= s->c.n_species || !flux || !mom) return ORC_EINVAL;
    int nn = s->nn;
    for (int i = 0; i < nn; ++i) { flux[i] = 0.0; mom[i] = 0.0; }
    for (int64_t p = 0; p < s->p[k].n; ++p) {
        int64_t c, c1;
        double f, vx = s->p[k].vx[p];
        locate(s, s->p[k].x[p], &c, &c1, &f);
        flux[c] += (1.0 - f) * vx;
        flux[c1] += f * vx;
        mom[c] += (1.0 - f) * vx * vx;
        mom[c1] += f * vx * vx;
    }
    for (int i = 0; i < nn; ++i) {
        flux[i] *= s->c.sp[k].weight / node_volume(s, i);
        mom[i] *= s->c.sp[k].weight / node_volume(s, i);
    }
    return ORC_OK;
}

int orc_get_counters(const orc_sim* s, orc_counters* out)
{
    if (!s || !out) return ORC_EINVAL;
    *out = s->cnt;
    return ORC_OK;
}

int orc_get_energy(const orc_sim* s, double* ke, double* fe)
{
    if (!s) return ORC_EINVAL;
    if (ke) for (int k = 0; k < s->c.n_species; ++k) ke[k] = s->ke[k];
    if (fe) *fe = s->fe;
    return ORC_OK;
}

int orc_get_numax(const orc_sim* s, int32_t k, double* numax, uint32_t* t32)
{
    if (!s || k < 0 || k >= s->c.n_species) return ORC_EINVAL;
    if (numax) *numax = s->numax[k];
    if (t32) *t32 = s->t32[k];
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Time-accumulated diagnostics (Section 1: densities, potential, mean
 * energies and energy distributions in the bulk and at the walls). */
int orc_set_diag(orc_sim* s, int32_t enable, double eepf_emax_ev)
{
    if (!s || !(eepf_emax_ev > 0.0)) return ORC_EINVAL;
    s->diag = enable ? 1 : 0;
    s->eepf_emax = eepf_emax_ev;
    return ORC_OK;
}

int orc_set_wall_edf(orc_sim* s, int32_t k, double emax_ev)
{
    if (!s || k < 0 || k >= s->c.n_species || !(emax_ev > 0.0)) return ORC_EINVAL;
    s->wedf_emax[k] = emax_ev;
    return ORC_OK;
}

int orc_reset_avg(orc_sim* s)
{
    if (!s) return ORC_EINVAL;
    for (int k = 0; k < s->c.n_species; ++k) {
        memset(s->av_dens[k], 0, (size_t)s->nn * sizeof(double));
        memset(s->av_pw[k], 0, (size_t)5 * s->nn * sizeof(double));
    }
    memset(s->av_phi, 0, (size_t)s->nn * sizeof(double));
    memset(s->av_neps, 0, (size_t)s->nn * sizeof(double));
    memset(s->eepf, 0, sizeof(s->eepf));
    memset(s->wedf, 0, sizeof(s->wedf));
    s->av_samples = 0.0;
    return ORC_OK;
}

int orc_get_avg(const orc_sim* s, double* out)
{
    if (!s || !out) return ORC_EINVAL;
    int nn = s->nn, S = s->c.n_species;
    double ns = s->av_samples;
    out[0] = ns;
    for (int k = 0; k < S; ++k)
        for (int i = 0; i < nn; ++i) out[1 + (size_t)k * nn + i] = ns > 0.0 ? s->av_dens[k][i] / ns : 0.0;
    for (int i = 0; i < nn; ++i) {
        out[1 + (size_t)S * nn + i] = ns > 0.0 ? s->av_phi[i] / ns : 0.0;
        double n = s->av_dens[0][i];
        out[1 + (size_t)(S + 1) * nn + i] = n > 0.0 ? s->av_neps[i] / n : 0.0;
    }
    return ORC_OK;
}

int orc_get_eepf(const orc_sim* s, double* out)
{
    if (!s || !out) return ORC_EINVAL;
    for (int w = 0; w < 2; ++w)
        for (int i = 0; i < ORC_EEPF_BINS; ++i) out[w * ORC_EEPF_BINS + i] = (double)s->eepf[w][i];
    out[2 * ORC_EEPF_BINS] = s->eepf_emax / ORC_EEPF_BINS;
    out[2 * ORC_EEPF_BINS + 1] = s->av_samples;
    return ORC_OK;
}

int orc_get_wall_edf(const orc_sim* s, double* out)
{
    if (!s || !out) return ORC_EINVAL;
    int S = s->c.n_species;
    for (int k = 0; k < S; ++k)
        for (int w = 0; w < 2; ++w)
            for (int i = 0; i < ORC_EEPF_BINS; ++i)
                out[((size_t)k * 2 + w) * ORC_EEPF_BINS + i] = (double)s->wedf[k][w][i];
    for (int k = 0; k < S; ++k) out[(size_t)S * 2 * ORC_EEPF_BINS + k] = s->wedf_emax[k] / ORC_EEPF_BINS;
    out[(size_t)S * 2 * ORC_EEPF_BINS + S] = s->av_samples;
    return ORC_OK;
}

int orc_get_circuit(const orc_sim* s, double out[2])
{
    if (!s || !out) return ORC_EINVAL;
    out[0] = s->phi[0];
    out[1] = s->qbase + q_source(s, (double)s->step * s->c.dt) + q_collected(s);
    return ORC_OK;
}

int orc_set_circuit(orc_sim* s, double q)
{
    if (!s || !isfinite(q) || !circuit_mode(s)) return ORC_EINVAL;
    s->qbase = q - q_source(s, (double)s->step * s->c.dt) - q_collected(s);
    s->circ_init = 1;
    return ORC_OK;
}
