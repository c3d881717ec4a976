// Internal layout of the MI355X PIC-MCC library: constant and mutable state of
// every (discharge, species) segment and of every discharge, and the kernel
// argument blocks.  Device memory is structure-of-arrays: per segment, one
// array per particle field (cell i32, in-cell offset f32, vx/vy/vz f32, id u32)
// in two copies: the step updates one copy in place, and the compaction of
// the holes left by absorbed particles (and the optional sort) writes the
// other, preserving the order of the live particles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"

namespace pic {

constexpr int kMaxSpecies = PIC_MAX_SPECIES;
constexpr int kMaxChan = PIC_MAX_CHAN;
constexpr int kMaxCells = 4096;
constexpr int kFinThreads = 1024;          // finalize / field-solve workgroup (4 nodes per thread at most)
constexpr int kNodesPerThread = 4;         // kFinThreads * 4 >= nodes of a bounded mesh
constexpr int kEepfBins = PIC_EEPF_BINS;
constexpr int kWindowRing = PIC_WINDOW_RING;
constexpr int kMaxSeg = PIC_MAX_BATCH * PIC_MAX_SPECIES;   // (discharge, species) segments of a context
constexpr int64_t kMaxTiles = 1ll << 30;                    // tile numbers fit in int32
constexpr int kTileMin = 256;                               // smallest tile of the push (particles)
constexpr int kBirthsDiv = 16;                              // a tile stages up to T / 16 births per step
constexpr int kBirthsPerTileMin = kTileMin / kBirthsDiv;
constexpr int kMaxPushGrid = 4096;                          // workgroups of a push launch
constexpr int kPow = 5;                                     // power time sums per species and node

// latched device flags
constexpr uint32_t kFlagCapacity = 1u << 0;
constexpr uint32_t kFlagNumeric = 1u << 1;
constexpr uint32_t kFlagNuMax = 1u << 2;
constexpr uint32_t kFlagCell = 1u << 3;
constexpr uint32_t kFlagStall = 1u << 4;

// Copies of the deposit accumulators and event counters: workgroup w adds into
// copy w % kRep, so no address takes more than 1/kRep of the atomics (device-
// scope atomics on one address serialise); readers sum the copies.
constexpr int kRep = 1;
// event counters per segment
enum { C_ABS0, C_ABS1, C_SEE0, C_SEE1, C_CAND, C_NULL, C_VIOL, C_DROP, C_REN, C_COLL, C_N = C_COLL + kMaxChan };

// Fixed-point scale of the deposit: a particle's weights (1-f, f) become the
// integers 2^32 - q and q, q = f * 2^32, so sums are exact and independent of
// the order in which tiles add them.
constexpr double kDepScale = 4294967296.0;

// a staged birth: the electron (ionization or secondary) and, for
// ionization, the velocity of the ion born with it; key = the parent's slot
// in its tile (births are staged in any order and ranked by key)
struct Birth {
    int32_t cell;
    float off, vx, vy, vz;
    float ivx, ivy, ivz;
    uint32_t key;
};

struct SegConst {
    // particle storage, [0] and [1] are the two copies (SegState::parity
    // says which holds the particles)
    int32_t* cell[2];
    float* off[2];
    float* vx[2];
    float* vy[2];
    float* vz[2];
    uint32_t* id[2];
    double* z[2];           // axial displacement since injection, FP64 (renewal only, else null)
    int64_t cap;
    // push
    float qmh;              // (q/m) dt/2
    float tv[3], sv[3];     // Boris rotation vectors t and s = 2t/(1+t^2)
    float dtdx;             // dt/dx
    float eext[3];          // imposed field
    double mw_half;         // m w / 2 (kinetic energy per unit area)
    double q, w, qm;
    float mass;
    int32_t compacts;       // 1 when particles can be absorbed (bounded domain)
    // collisions: the candidate test in the push, the rest (channel,
    // kinematics, births) in the events kernel, in FP64
    int32_t nch, ion_type;
    uint32_t t32;
    int32_t xs_n;
    double xs_ln0, xs_inv_dln;
    const double* xs;       // [xs_n][nch] n_g sigma_k / nu_max on a uniform ln(eps) grid
    int32_t kind[kMaxChan];
    double th[kMaxChan];
    float half_m_over_e;    // m / 2e in FP32 (wall energies, diagnostics)
    double half_m_over_e_d, two_e_over_m;
    double mr2;             // 2 m / M_gas
    double vt_gas;          // sqrt(k T_g / M_gas)
    double m_frac, M_frac;  // m/(m+M), M/(m+M)
    // secondary emission by this (ion) species
    int32_t emits;
    uint32_t see_k;         // emit iff (2*(x>>9)+1) < see_k
    double vsee;            // sqrt(e T_see / m_e)
    double dtdx_e;          // dt/dx of the electron species (same mesh and dt)
    // velocity moments (diagnostics) in fixed point: per particle weight x
    // vx x mscale1 and weight x vx^2 x mscale2, rounded to integers
    float mscale1, mscale2;
    float wedf_inv_bin;     // wall impact-energy histogram: 1 / bin width (1/eV)
    // axial renewal: length (0 = off) and dt, the initial distribution
    double renew_lz, dt_d;
    double vth0;
    double drift0[3];
};

struct DisConst {
    int32_t n_cells, n_nodes, bc, field_solve;
    double dx, dt, L, eps0, rho_bg, v_amp, v_freq, v_phase;
    double e_ext[3], b_ext[3];
    double c2;                 // dx^2 / eps0
    double inv_2dx, inv_dx;
    double wall_coef;          // dx / (2 eps0)
    double dens_coef[kMaxSpecies];   // weight / dx / 2^32 (interior node; twice at a wall node)
    double q[kMaxSpecies];     // species charge
    double flux_coef[kMaxSpecies], mom_coef[kMaxSpecies];   // moment sums -> densities (interior node)
    double mass[kMaxSpecies];  // species mass (power decomposition)
    uint32_t key0, key1;
    int32_t bulk_lo, bulk_hi;  // cells of the bulk electron energy distribution
    // drive of the electrode at x = 0
    int32_t drive, waveform;
    double cap, j_amp;
    double qw[kMaxSpecies];    // charge x weight of a macro-particle, C/m^2
};

// mutable, one per segment.  Slots [0, count) hold the particles in their
// canonical order, with holes (cell < 0) where particles were absorbed since
// the last compaction; births are appended after the last slot.
struct SegState {
    int64_t count;          // slots in use (live particles and holes)
    int64_t live;           // live particles
    int64_t dead;           // particles absorbed in the current step
    int64_t staged;         // births staged by this segment's tiles in the current step
    int64_t tile_first, ntiles;  // tile range of the current step (tiles are numbered over all segments)
    uint32_t next_id;
    int32_t parity;         // which copy holds the particles
    double ke;              // time-centred kinetic energy of the last step
};

// mutable, one per discharge
struct DisState {
    uint64_t step;
    uint32_t flags;
    int32_t retired;        // non-zero: skipped by the step kernels
    double fe;
    double avg_samples;
    double eepf_samples;
    double qbase;           // circuit: conductor charge minus the source's and the particles' since the start
    int32_t circ_init;      // circuit: qbase set
    int64_t win_len, win_start, nwin;   // RF windows: length in steps (0 = off), first step, windows done
    uint64_t pw_next;       // power decomposition: the step whose previous flux is stored (else none)
};

// The source of the electrode at x = 0: its voltage V(t), and the charge per
// area a current source has delivered since t = 0 (the integral of
// j_amp sin(w t + phase)).
__host__ __device__ inline double source_voltage(const DisConst& dc, double t)
{
    const double w = 6.283185307179586476925286766559 * dc.v_freq;
    if (dc.waveform == PIC_WAVE_TWO_HARMONIC) return dc.v_amp * (cos(w * t + dc.v_phase) + cos(2.0 * w * t));
    return dc.v_amp * sin(w * t + dc.v_phase);
}

__host__ __device__ inline double source_charge(const DisConst& dc, double t)
{
    if (dc.drive != PIC_DRIVE_CURRENT) return 0.0;
    const double w = 6.283185307179586476925286766559 * dc.v_freq;
    return dc.j_amp / w * (cos(dc.v_phase) - cos(w * t + dc.v_phase));
}

// Charge per area particles have brought to the electrode at x = 0, from the
// event counters [S][kRep][C_N] of one discharge: absorbed particles bring
// theirs, each secondary electron emitted there takes one away.
__host__ __device__ inline double collected_charge(const DisConst& dc, const unsigned long long* cnt, int S)
{
    double q = 0.0;
    unsigned long long see = 0ull;
    for (int s = 0; s < S; ++s) {
        unsigned long long ab = 0ull;
        for (int r = 0; r < kRep; ++r) {
            ab += cnt[((size_t)s * kRep + r) * C_N + C_ABS0];
            see += cnt[((size_t)s * kRep + r) * C_N + C_SEE0];
        }
        q += dc.qw[s] * (double)ab;
    }
    return q - dc.qw[0] * (double)see;
}

struct Ctx;  // host

struct DevPtrs {
    int32_t B, S;
    SegConst* segc;              // [B*S]
    SegState* segs;              // [B*S]
    DisConst* disc;              // [B]
    DisState* diss;              // [B]
    unsigned long long* acc;     // [B][S][kRep][nodes_max] deposit sums (fixed point)
    unsigned long long* cnt;     // [B][S][kRep][C_N] event counters
    unsigned long long* eacc;    // [B][nodes_max] electron energy deposit (eV, fixed point 2^20)
    unsigned long long* macc;    // [B][S][2][nodes_max] flux and x-momentum flux sums of the step (fixed point)
    double* pavg;                // [B][S][kPow][nodes_max] time sums: flux, momentum flux, power density,
                                 // inertia and pressure terms of the power decomposition
    double* gprev;               // [B][S][nodes_max] the flux of the last sampled step
    double* ptmp;                // [B][2][nodes_max] node scratch of the decomposition's gradients
    unsigned long long* wen;     // [B][S][2] kinetic energy carried into each wall (eV, fixed point 2^20)
    double* rho;                 // [B][nodes_max]
    double* phi;
    double* ef;
    double* dens;                // [B][S][nodes_max]
    float2* epair;               // [B][cells_max] (E[c], E[c+1]) for the gather
    double* avg;                 // [B][(S+2)][nodes_max]
    unsigned long long* eepf;    // [B][2][bins]
    double* wring;               // [B][kWindowRing][1 + (S+2) nodes_max] completed windows: samples, sums as avg
    unsigned long long* wedf;    // [B][S][2][bins] impact energies at each wall
    Birth* births;               // [tiles_max * kBirthsPerTileMin] births staged by tile, in particle order
    int32_t* bcnt;               // [tiles_max] births staged by each tile
    uint4* evr;                  // [slots] events of the step, packed per push workgroup from the first slot
                                 // of its tile range, in any order: (slot in tile | event bits, id, vx, vy)
                                 // of the particle after the push
    uint4* evq;                  // [slots] the same events' (vz, cell, offset, tile)
    uint32_t* evg;               // [kMaxPushGrid] events of each push workgroup's range
    unsigned long long* tick;    // steps taken by the context
    uint32_t* ccnt;              // [tiles_max] compaction: live particles of each tile, then their first slot
    double* ke_part;             // [tiles_max] kinetic-energy partial sums by tile
    int32_t nodes_max, cells_max;
    int64_t tiles_max;
};

}  // namespace pic
