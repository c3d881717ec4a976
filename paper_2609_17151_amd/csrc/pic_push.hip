// Particle kernels of one leapfrog step for every species of every discharge
// of a context (paper Section 1: explicit leapfrog, Boris pusher, walls and
// secondary emission, null-collision Monte Carlo with tabulated cross
// sections; the charge of the particles deposited on the mesh).
//
// The push is one launch over all segments.  Work is cut into tiles of
// T = threads * PPT consecutive particle slots of one (discharge, species)
// segment; tiles are numbered over all segments, discharge-major, and every
// workgroup takes a fixed contiguous range of tiles, so no workgroup ever
// waits for another.  Each thread owns PPT consecutive slots and moves them
// with 16-byte vector loads and stores, in place.  A workgroup stages the
// (E[c], E[c+1]) pairs of a discharge in LDS once per run of tiles of that
// discharge, and zeroes and flushes its deposit histogram once per run of
// tiles of one segment.
//
// Per particle the push does the gather (linear weighting), the Boris push in
// the imposed B, the cell-relative move in FP32, the periodic wrap or the
// absorption at a wall, and the null-collision candidate test (an integer
// test on one Philox draw).  What only a few particles need per step is
// recorded as an event instead: a collision candidate, an axial renewal, the
// secondary-emission test of an absorbed ion.  Each wave appends its events'
// records to its workgroup's packed list at a place one LDS atomic claims
// (ballots and lane counts: no barrier, no queue); the events pass then does
// that work for all of them with full waves, in FP64: in the events kernel,
// or at the end of each push workgroup for its own list (FUSE).
//
// Absorbed particles leave holes (cell = -1) that later steps skip; a stable
// compaction every few steps removes them.  Holes do not change the order of
// the live particles, and births are appended after the last slot in the
// order of their parents, so the particle order after a compaction is the
// order that compacting every step would give.  The events pass stages a
// tile's births in any order, each with a key made of its parent's slot and
// its rank among that parent's births; the finalize writes each birth at the
// rank of its key within its tile, the tiles in order, which also gives their
// ids.
//
// Deposition: LDS histogram in 64-bit fixed point flushed with integer
// atomics (births add theirs with integer atomics too), so sums are exact and
// independent of the order of tiles and runs are bit-reproducible without
// global float atomics.
//
// Streaming instances (GENERAL = false) serve periodic runs without
// collisions or renewal, where nothing can be absorbed or born: no ids,
// holes or events.
#include "pic_device.h"
#include "pic_internal.h"
#include "pic_kernels.h"

namespace pic {

namespace {

__device__ __forceinline__ void lds_deposit(unsigned long long* hist, int c, float f, int n_cells,
                                            int periodic)
{
    uint32_t q = (uint32_t)(f * 4294967296.0f);
    if (f >= 1.0f) q = 0xFFFFFFFFu;
    const int c1 = (periodic && c + 1 == n_cells) ? 0 : c + 1;
    atomicAdd(&hist[c], (unsigned long long)(0x100000000ull - q));
    atomicAdd(&hist[c1], (unsigned long long)q);
}

__device__ __forceinline__ void global_deposit(unsigned long long* acc, int c, float f, int n_cells,
                                               int periodic)
{
    uint32_t q = (uint32_t)(f * 4294967296.0f);
    if (f >= 1.0f) q = 0xFFFFFFFFu;
    const int c1 = (periodic && c + 1 == n_cells) ? 0 : c + 1;
    atomicAdd(&acc[c], (unsigned long long)(0x100000000ull - q));
    atomicAdd(&acc[c1], (unsigned long long)q);
}

// Particle arrays are device global memory.  Reaching them through
// address-space-1 pointers lets the compiler use global instead of flat
// memory instructions (measured 8 % faster on the streaming push).
#define PIC_GLOBAL __attribute__((address_space(1)))

// NT: non-temporal (streaming) accesses, which leave the caches to the rest
// of the step.  Measured on the 64-discharge argon sweep (4.7e7 particles):
// the general push 541 -> 461 us (each at its fastest tile shape) and the
// events kernel after it 97 -> 80 us.  The streaming push on the E x B box,
// whose particle arrays fit the Infinity Cache between steps, is 11 % slower
// with them and does not use them.
template <int N, typename V, bool NT = false, typename S>
__device__ __forceinline__ void vload(const S* __restrict__ p, S* out)
{
    if constexpr (N % 4 == 0) {
        typedef S NV __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int k = 0; k < N / 4; ++k) {
            const PIC_GLOBAL NV* q = (const PIC_GLOBAL NV*)(p) + k;
            const NV v = NT ? __builtin_nontemporal_load(q) : *q;
            out[4 * k + 0] = v.x;
            out[4 * k + 1] = v.y;
            out[4 * k + 2] = v.z;
            out[4 * k + 3] = v.w;
        }
    } else {                       // (2-wide vector loads measured 4 % slower here)
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const PIC_GLOBAL S* q = (const PIC_GLOBAL S*)(p) + k;
            out[k] = NT ? __builtin_nontemporal_load(q) : *q;
        }
    }
}

template <int N, typename V, bool NT = false, typename S>
__device__ __forceinline__ void vstore(S* __restrict__ p, const S* in)
{
    if constexpr (N % 4 == 0) {
        typedef S NV __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int k = 0; k < N / 4; ++k) {
            NV v;
            v.x = in[4 * k + 0];
            v.y = in[4 * k + 1];
            v.z = in[4 * k + 2];
            v.w = in[4 * k + 3];
            PIC_GLOBAL NV* q = (PIC_GLOBAL NV*)(p) + k;
            if (NT)
                __builtin_nontemporal_store(v, q);
            else
                *q = v;
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            PIC_GLOBAL S* q = (PIC_GLOBAL S*)(p) + k;
            if (NT)
                __builtin_nontemporal_store(in[k], q);
            else
                *q = in[k];
        }
    }
}

// Events of the step, recorded by the push for the events pass: the slot
// of the particle in its tile and what happens to it there.
constexpr uint32_t kEvSlot = 0xffffu;       // slot in the tile (tiles hold at most 4096 particles)
constexpr uint32_t kEvCand = 1u << 16;      // collision candidate
constexpr uint32_t kEvRenew = 1u << 17;     // axial renewal: a fresh velocity
constexpr uint32_t kEvSee = 1u << 18;       // an emitting ion absorbed at a wall: secondary emission test
constexpr uint32_t kEvWall1 = 1u << 19;     // ... at the wall x = L
constexpr int kEvSegShift = 20;             // the particle's segment (kMaxSeg <= 1024: 10 bits)
static_assert(kMaxSeg <= 1024, "the event word holds the segment in 10 bits");
static_assert(C_N <= 64, "the flush's counters are held by one wave's lanes");

// The constants of a tile's segment that the particle loop reads, copied to
// registers once per tile.  The segment index is made wave-uniform, so these
// are scalar loads; read through the segment's structure instead, every
// particle would reload them, since the loop's atomics could alias them.
struct PushC {
    int nc, periodic, emits, nch;
    uint32_t t32, key0, key1;
    float ex, ey, ez, qmh, tx, ty, tz, sx, sy, sz, dtdx, hme, wedf_inv_bin, mscale1, mscale2;
    int bulk_lo, bulk_hi;
};

__device__ __forceinline__ PushC push_consts(const SegConst& sc, const DisConst& dc)
{
    PushC k;
    k.nc = dc.n_cells;
    k.periodic = dc.bc == PIC_BC_PERIODIC;
    k.emits = sc.emits;
    k.nch = sc.nch;
    k.t32 = sc.t32;
    k.key0 = dc.key0;
    k.key1 = dc.key1;
    k.ex = sc.eext[0];
    k.ey = sc.eext[1];
    k.ez = sc.eext[2];
    k.qmh = sc.qmh;
    k.tx = sc.tv[0];
    k.ty = sc.tv[1];
    k.tz = sc.tv[2];
    k.sx = sc.sv[0];
    k.sy = sc.sv[1];
    k.sz = sc.sv[2];
    k.dtdx = sc.dtdx;
    k.hme = sc.half_m_over_e;
    k.wedf_inv_bin = sc.wedf_inv_bin;
    k.mscale1 = sc.mscale1;
    k.mscale2 = sc.mscale2;
    k.bulk_lo = dc.bulk_lo;
    k.bulk_hi = dc.bulk_hi;
    return k;
}

// A particle's step in the push: gather, Boris push, cell-relative move,
// periodic wrap or absorption, and the collision test.  Returns whether the
// particle stays; `ev` collects its event bits (the collision itself, the
// secondary emission and the renewal are the events pass's).
template <bool GENERAL>
__device__ __forceinline__ bool advance(const DevPtrs& d, const PushC& k, const PushArgs& a, int s, int b,
                                        uint32_t step, const float2* ep, unsigned int* s_cnt,
                                        unsigned long long* s_wen, int& c, float& f, float& ux, float& uy,
                                        float& uz, uint32_t pid, float& ke_sum, uint32_t& ev)
{
    const int nc = k.nc;
    if ((unsigned)c >= (unsigned)nc) {     // corrupt state: latch, park the particle
        atomicOr(&d.diss[b].flags, kFlagCell);
        c = 0;
        f = 0.0f;
    }
    // gather
    const float2 e2 = ep[c];
    const float ex = e2.x + f * (e2.y - e2.x) + k.ex;
    const float ey = k.ey, ez = k.ez;
    // Boris: half kick, rotation, half kick
    const float qmh = k.qmh;
    const float tx = k.tx, ty = k.ty, tz = k.tz;
    const float sx = k.sx, sy = k.sy, sz = k.sz;
    const float vold2 = ux * ux + uy * uy + uz * uz;
    ux += qmh * ex;
    uy += qmh * ey;
    uz += qmh * ez;
    const float px = ux + (uy * tz - uz * ty);
    const float py = uy + (uz * tx - ux * tz);
    const float pz = uz + (ux * ty - uy * tx);
    ux += py * sz - pz * sy;
    uy += pz * sx - px * sz;
    uz += px * sy - py * sx;
    ux += qmh * ex;
    uy += qmh * ey;
    uz += qmh * ez;
    const float vnew2 = ux * ux + uy * uy + uz * uz;
    ke_sum += vold2 + vnew2;
    // move, relative to the cell
    f += ux * k.dtdx;
    const float fl = floorf(f);
    c += (int)fl;
    f -= fl;
    if (f >= 1.0f) {
        f -= 1.0f;
        c += 1;
    }
    if (!(f >= 0.0f && f < 1.0f) || !(fabsf(ux) < 3.0e38f)) {   // non-finite state
        atomicOr(&d.diss[b].flags, kFlagNumeric);
        f = 0.0f;
        c = 0;
        ux = uy = uz = 0.0f;
    }
    if (k.periodic) {
        if (c < 0) c += nc;
        else if (c >= nc) c -= nc;
        if ((unsigned)c >= (unsigned)nc) {                     // moved more than the domain
            atomicOr(&d.diss[b].flags, kFlagCell);
            c = 0;
            f = 0.0f;
        }
        if (!GENERAL) return true;
    } else if (c < 0 || c >= nc) {
        const int wall = c < 0 ? 0 : 1;
        atomicAdd(&s_cnt[C_ABS0 + wall], 1u);
        atomicAdd(&s_wen[wall], (unsigned long long)(k.hme * vnew2 * 1048576.0f));
        if (a.diag) {
            // impact energy: this species' histogram at this wall, and for
            // electrons the wall energy distribution
            const float eps = k.hme * vnew2;
            const int wb = (int)(eps * k.wedf_inv_bin);
            if ((unsigned)wb < (unsigned)kEepfBins)
                atomicAdd(&d.wedf[(((size_t)b * d.S + s) * 2 + wall) * kEepfBins + wb], 1ull);
            const int bin = (int)(eps * a.eepf_inv_bin);
            if (s == 0 && (unsigned)bin < (unsigned)kEepfBins)
                atomicAdd(&d.eepf[((size_t)b * 2 + 1) * kEepfBins + bin], 1ull);
        }
        if (GENERAL && k.emits) ev = kEvSee | (wall ? kEvWall1 : 0u);
        return false;
    }
    if (!GENERAL || k.nch == 0) return true;
    // null-collision Monte Carlo: integer candidate test on the first draw
    const uint4 r = philox10(pid, step, ((uint32_t)s << 24), 0u, k.key0, k.key1);
    if (r.x < k.t32) ev |= kEvCand;
    return true;
}

// velocity moments of a particle at the nodes, fixed point (diagnostics);
// fh and mh are LDS histograms in the push and the discharge's global sums
// in the events pass; ms1, ms2 the species' fixed-point scales
__device__ __forceinline__ void moment_diag(float ms1, float ms2, unsigned long long* fh, unsigned long long* mh,
                                            int c, float f, float ux, int nc, int periodic)
{
    const int c1 = (periodic && c + 1 == nc) ? 0 : c + 1;
    const float a = ux * ms1, b2 = ux * ux * ms2;
    const float w0 = 1.0f - f;
    atomicAdd(&fh[c], (unsigned long long)(long long)rintf(w0 * a));
    atomicAdd(&fh[c1], (unsigned long long)(long long)rintf(f * a));
    atomicAdd(&mh[c], (unsigned long long)(long long)rintf(w0 * b2));
    atomicAdd(&mh[c1], (unsigned long long)(long long)rintf(f * b2));
}

// electron energy at the nodes and in the bulk distribution (diagnostics);
// CT is the bin counter type (32-bit in LDS, 64-bit in global memory); hme =
// m / 2e, [lo, hi) the cells of the bulk distribution
template <typename CT>
__device__ __forceinline__ void electron_diag(float hme, int lo, int hi, float eepf_inv_bin,
                                              unsigned long long* ehist, CT* eepf, int c, float f,
                                              float ux, float uy, float uz, int nc, int periodic)
{
    const float eps = hme * (ux * ux + uy * uy + uz * uz);
    const float w1 = f * eps, w0 = eps - w1;
    const int c1 = (periodic && c + 1 == nc) ? 0 : c + 1;
    atomicAdd(&ehist[c], (unsigned long long)(w0 * 1048576.0f));
    atomicAdd(&ehist[c1], (unsigned long long)(w1 * 1048576.0f));
    if (c >= lo && c < hi) {
        const int bin = (int)(eps * eepf_inv_bin);
        if ((unsigned)bin < (unsigned)kEepfBins) atomicAdd(&eepf[bin], (CT)1);
    }
}

// block reduction in a fixed order (deterministic)
template <int BS>
__device__ __forceinline__ double block_sum_f32(float v, float* s_w)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const float w = wave_sum_f32(v);
    __syncthreads();
    if (lane == 0) s_w[wid] = w;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < BS / 64; ++k) t += (double)s_w[k];
    return t;
}

// First tile of every (discharge, species) segment for tiles of T particles,
// from the device-resident counts (retired discharges get none): s_pref[g]
// is the first tile of segment g, s_pref[NS] the number of tiles.  Wave 0,
// up to 16 segments per lane; the caller synchronises.
__device__ __forceinline__ void tile_prefix(const DevPtrs& d, int T, int32_t* s_pref)
{
    const int S = d.S, NS = d.B * d.S;
    const int lane = threadIdx.x & 63;
    if ((threadIdx.x >> 6) != 0) return;
    const int per = (NS + 63) >> 6;
    const int g0 = lane * per;
    int32_t run = 0;
    for (int j = 0; j < per; ++j) {
        const int g = g0 + j;
        if (g < NS) {
            const int64_t n = d.diss[g / S].retired ? 0 : d.segs[g].count;
            run += (int32_t)((n + T - 1) / T);
            s_pref[g + 1] = run;
        }
    }
    int32_t incl = run;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
        const int32_t o = __shfl_up(incl, dd, 64);
        if (lane >= dd) incl += o;
    }
    const int32_t excl = incl - run;
    if (lane == 0) s_pref[0] = 0;
    for (int j = 0; j < per; ++j) {
        const int g = g0 + j;
        if (g < NS) s_pref[g + 1] += excl;
    }
}

// the segment of tile t: the last g with s_pref[g] <= t
__device__ __forceinline__ int tile_segment(const int32_t* s_pref, int NS, int32_t t)
{
    int lo = 0, hi = NS;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_pref[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

}  // namespace

// The events pass over one chunk of 64 events of a push workgroup's list,
// one event per lane (defined with the events kernel below): the records of
// the chunk, then the work on them.
struct EvPass {
    int32_t T;                    // particles of the push's tile
    int32_t chunk_t, NT;          // tiles per push workgroup, tiles in all
    uint32_t bpt;                 // births staged per tile at most
    int32_t diag;
    float eepf_inv_bin;
};

__device__ __forceinline__ bool event_record(const DevPtrs& d, const EvPass& ps, int g, uint32_t nev, uint32_t kc,
                                             uint4& rec, uint4& rq);
__device__ __forceinline__ void event_chunk(const DevPtrs& d, const int32_t* s_pref, int NS, const EvPass& ps,
                                            bool act, uint4 rec, uint4 rq);

// FUSE: the workgroup does its own tile range's events after its push (no
// events launch; for workloads too small to fill the GPU twice)
template <int PPT, int BS, bool GENERAL, bool FUSE>
__global__ __launch_bounds__(BS) void push_kernel(PushArgs a)
{
    constexpr int kBS = BS;
    constexpr int T = kBS * PPT;
    constexpr int kWavesPerTile = kBS / 64;
    const DevPtrs& d = a.d;
    const int S = d.S, NS = d.B * d.S;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t s_pref[kMaxSeg + 1];   // first tile of every segment (discharge-major)
    __shared__ unsigned int s_cnt[C_N];
    __shared__ unsigned long long s_wen[2];   // energy carried into each wall by the run (eV, 2^20)
    __shared__ float s_red[kBS / 64];
    __shared__ uint32_t s_evn;                // events recorded by the workgroup

    tile_prefix(d, T, s_pref);
    if (tid < C_N) s_cnt[tid] = 0;
    if (tid < 2) s_wen[tid] = 0ull;
    if (tid == 0) s_evn = 0u;
    __syncthreads();
    const int32_t NT = s_pref[NS];

    // LDS layout: deposit histogram, [energy, flux and momentum-flux
    // histograms, EEPF], E pairs
    const int nn_max = a.nodes_max_dyn;
    const int dn = a.diag ? nn_max : 0;
    unsigned long long* hist = reinterpret_cast<unsigned long long*>(smem);
    unsigned long long* ehist = hist + nn_max;
    unsigned long long* fhist = ehist + dn;
    unsigned long long* mhist = fhist + dn;
    unsigned int* eepf = reinterpret_cast<unsigned int*>(mhist + dn);
    float2* ep = reinterpret_cast<float2*>(eepf + (a.diag ? kEepfBins : 0));

    int cur_g = -1, cur_b = -1;
    int32_t run_first = 0;
    float ke_run = 0.0f;
    // the current segment's particle arrays and counts, read when the segment
    // changes, so that a tile's particle loads do not wait for them
    int64_t n = 0;
    uint32_t step = 0;
    int32_t tile_first = 0, ntiles = 0;
    int32_t* p_cell = nullptr;
    float *p_off = nullptr, *p_vx = nullptr, *p_vy = nullptr, *p_vz = nullptr;
    uint32_t* p_id = nullptr;
    double* p_z = nullptr;
    double renew_lz = 0.0, dt_d = 0.0;
    // a fixed contiguous range of tiles per workgroup
    const int32_t chunk = (NT + (int32_t)gridDim.x - 1) / (int32_t)gridDim.x;
    const int32_t t_begin = (int32_t)blockIdx.x * chunk;
    const int32_t t_end = t_begin + chunk < NT ? t_begin + chunk : NT;

    // flush the run of tiles of segment cg: deposit, diagnostics, counters,
    // kinetic energy (ranges are fixed, so the grouping of the sums is too).
    // The first `quiet` threads (whole waves) take part in the barriers only,
    // so that no memory operation of the flush is outstanding in those waves
    // when they go on to the events pass.
    auto flush = [&](int cg, int quiet) {
        __syncthreads();
        const int ft = tid - quiet, nt = kBS - quiet;
        const int cb = cg / S, cs = cg - cb * S;
        const DisConst& dcf = d.disc[cb];
        const int rep = blockIdx.x % kRep;
        if (ft >= 0) {
            unsigned long long* acc_s = d.acc + ((size_t)cg * kRep + rep) * d.nodes_max;
            for (int i = ft; i < dcf.n_nodes; i += nt) {
                const unsigned long long v = hist[i];
                if (v) atomicAdd(&acc_s[i], v);
            }
            if (a.diag) {
                unsigned long long* ma = d.macc + (size_t)cg * 2 * d.nodes_max;
                for (int i = ft; i < dcf.n_nodes; i += nt) {
                    const unsigned long long v = fhist[i], w = mhist[i];
                    if (v) atomicAdd(&ma[i], v);
                    if (w) atomicAdd(&ma[d.nodes_max + i], w);
                }
            }
            if (a.diag && cs == 0) {
                unsigned long long* ea = d.eacc + (size_t)cb * d.nodes_max;
                for (int i = ft; i < dcf.n_nodes; i += nt) {
                    const unsigned long long v = ehist[i];
                    if (v) atomicAdd(&ea[i], v);
                }
                unsigned long long* eg = d.eepf + (size_t)cb * 2 * kEepfBins;
                for (int i = ft; i < kEepfBins; i += nt) {
                    const unsigned int v = eepf[i];
                    if (v) atomicAdd(&eg[i], (unsigned long long)v);
                }
            }
            unsigned long long* cnt = d.cnt + ((size_t)cg * kRep + rep) * C_N;
            if (ft < C_N) {
                const unsigned int v = s_cnt[ft];
                if (v) {
                    atomicAdd(&cnt[ft], (unsigned long long)v);
                    if (ft == C_ABS0 || ft == C_ABS1)
                        atomicAdd(reinterpret_cast<unsigned long long*>(&d.segs[cg].dead), (unsigned long long)v);
                }
                s_cnt[ft] = 0;
            }
            if (ft < 2) {
                const unsigned long long v = s_wen[ft];
                if (v) atomicAdd(&d.wen[(size_t)cg * 2 + ft], v);
                s_wen[ft] = 0ull;
            }
        }
        if (a.diag) {
            const double kt = block_sum_f32<BS>(ke_run, s_red);
            if (ft == 0) d.ke_part[run_first] = 0.5 * d.segc[cg].mw_half * kt;
            ke_run = 0.0f;
        }
    };

    // the tile's segment, wave-uniform (its constants become scalar loads):
    // found once, then followed along the workgroup's contiguous range
    int sg_walk = t_begin < t_end ? tile_segment(s_pref, NS, t_begin) : 0;
    for (int32_t t = t_begin; t < t_end; ++t) {
        while (s_pref[sg_walk + 1] <= t) ++sg_walk;
        const int sg = __builtin_amdgcn_readfirstlane(sg_walk);
        const int b = sg / S, s = sg - b * S;
        const DisConst& dc = d.disc[b];
        if (sg != cur_g) {
            if (cur_g >= 0) flush(cur_g, 0);
            __syncthreads();
            if (b != cur_b) {
                const float2* epg = d.epair + (size_t)b * d.cells_max;
                for (int i = tid; i < dc.n_cells; i += kBS) ep[i] = epg[i];
            }
            for (int i = tid; i < dc.n_nodes; i += kBS) hist[i] = 0ull;
            if (a.diag) {
                for (int i = tid; i < dc.n_nodes; i += kBS) {
                    fhist[i] = 0ull;
                    mhist[i] = 0ull;
                }
            }
            if (a.diag && s == 0) {
                for (int i = tid; i < dc.n_nodes; i += kBS) ehist[i] = 0ull;
                for (int i = tid; i < kEepfBins; i += kBS) eepf[i] = 0u;
            }
            cur_g = sg;
            cur_b = b;
            run_first = t;
            const SegConst& sc = d.segc[sg];
            const SegState& st = d.segs[sg];
            const int io = st.parity;             // updated in place
            n = st.count;
            step = (uint32_t)d.diss[b].step;
            tile_first = __builtin_amdgcn_readfirstlane(s_pref[sg]);
            ntiles = __builtin_amdgcn_readfirstlane(s_pref[sg + 1]) - tile_first;
            p_cell = sc.cell[io];
            p_off = sc.off[io];
            p_vx = sc.vx[io];
            p_vy = sc.vy[io];
            p_vz = sc.vz[io];
            p_id = sc.id[io];
            p_z = sc.z[io];
            renew_lz = sc.renew_lz;
            dt_d = sc.dt_d;
            __syncthreads();
        }
        const int32_t tin = t - tile_first;
        const PushC k = push_consts(d.segc[sg], dc);   // loads in flight with the particles'
        const int nc = k.nc;
        const int periodic = k.periodic;
        const int64_t base = (int64_t)tin * T + (int64_t)tid * PPT;

        int32_t cell[PPT];
        float off[PPT], vx[PPT], vy[PPT], vz[PPT];
        uint32_t pid[PPT];
        vload<PPT, int4, GENERAL>(p_cell + base, cell);
        vload<PPT, float4, GENERAL>(p_off + base, off);
        vload<PPT, float4, GENERAL>(p_vx + base, vx);
        vload<PPT, float4, GENERAL>(p_vy + base, vy);
        vload<PPT, float4, GENERAL>(p_vz + base, vz);
        if (GENERAL) {
            vload<PPT, uint4, GENERAL>(p_id + base, pid);
        } else {
#pragma unroll
            for (int j = 0; j < PPT; ++j) pid[j] = 0u;
        }
        // axial renewal: the displacement along the third axis since
        // injection, summed in FP64 (a slow ion adds only a few binary32
        // spacings of z per step, so a binary32 sum would drift)
        const bool renews = GENERAL && renew_lz > 0.0;
        double zax[PPT];
        if (renews) {
#pragma unroll
            for (int j = 0; j < PPT; ++j) zax[j] = p_z[base + j];
        }

        uint32_t evw[PPT];
        float ke_tile = 0.0f;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            evw[j] = 0u;
            if (base + j >= n) continue;
            if (GENERAL && cell[j] < 0) continue;          // a hole: absorbed earlier
            const bool keep = advance<GENERAL>(d, k, a, s, b, step, ep, s_cnt, s_wen, cell[j], off[j], vx[j], vy[j],
                                               vz[j], pid[j], ke_tile, evw[j]);
            if (renews && keep) {
                // past L_z the particle gets a fresh velocity from its
                // species' initial distribution at the same x (events pass)
                const double zz = zax[j] + (double)vz[j] * dt_d;
                if (fabs(zz) >= renew_lz) {
                    evw[j] |= kEvRenew;
                    zax[j] = 0.0;
                    atomicAdd(&s_cnt[C_REN], 1u);
                } else {
                    zax[j] = zz;
                }
            }
            if (keep) {
                lds_deposit(hist, cell[j], off[j], nc, periodic);
                // a particle whose velocity the events pass changes is
                // sampled there
                if (a.diag && !(evw[j] & (kEvCand | kEvRenew))) {
                    moment_diag(k.mscale1, k.mscale2, fhist, mhist, cell[j], off[j], vx[j], nc, periodic);
                    if (s == 0)
                        electron_diag(k.hme, k.bulk_lo, k.bulk_hi, a.eepf_inv_bin, ehist, eepf, cell[j], off[j],
                                      vx[j], vy[j], vz[j], nc, periodic);
                }
            } else {
                cell[j] = -1;                              // absorbed: leaves a hole
            }
        }
        ke_run += ke_tile;

        // in place; every particle keeps its slot
        if (base + PPT <= n) {
            vstore<PPT, int4, GENERAL>(p_cell + base, cell);
            vstore<PPT, float4, GENERAL>(p_off + base, off);
            vstore<PPT, float4, GENERAL>(p_vx + base, vx);
            vstore<PPT, float4, GENERAL>(p_vy + base, vy);
            vstore<PPT, float4, GENERAL>(p_vz + base, vz);
        } else {
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                if (base + j < n) {
                    p_cell[base + j] = cell[j];
                    p_off[base + j] = off[j];
                    p_vx[base + j] = vx[j];
                    p_vy[base + j] = vy[j];
                    p_vz[base + j] = vz[j];
                }
            }
        }
        if (renews) {
#pragma unroll
            for (int j = 0; j < PPT; ++j)
                if (base + j < n) p_z[base + j] = zax[j];
        }
        if (GENERAL) {
            // this wave's events, appended to the workgroup's packed list at
            // a place one LDS atomic per wave claims (no barrier): the order
            // of the records does not matter, each is self-contained and
            // every result of the events pass is independent of it
            uint32_t below = 0, total = 0;
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const uint64_t m = __ballot(evw[j] != 0u);
                below += lanes_below(m);
                total += (uint32_t)__popcll(m);
            }
            if (total) {
                uint32_t wbase = 0;
                if (lane == 0) wbase = atomicAdd(&s_evn, total);
                wbase = (uint32_t)__builtin_amdgcn_readfirstlane((int)wbase);
                // the particle after the push: slot, event bits, id, velocity,
                // position and tile, so the events pass reads the record only
                const size_t r0 = (size_t)t_begin * T + wbase;
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    if (evw[j]) {
                        d.evr[r0 + below] = make_uint4(evw[j] | (uint32_t)(tid * PPT + j) |
                                                           ((uint32_t)sg << kEvSegShift),
                                                       pid[j], __float_as_uint(vx[j]), __float_as_uint(vy[j]));
                        d.evq[r0 + below] = make_uint4(__float_as_uint(vz[j]), (uint32_t)cell[j],
                                                       __float_as_uint(off[j]), (uint32_t)t);
                        ++below;
                    }
                }
            }
        }
        if (tid == 0 && tin == ntiles - 1) {
            d.segs[sg].tile_first = tile_first;
            d.segs[sg].ntiles = ntiles;
        }
        if (GENERAL && tid == 0) d.bcnt[t] = 0;   // the events pass counts this tile's births
    }
    if (!GENERAL) {
        if (cur_g >= 0) flush(cur_g, 0);
        return;
    }
    __syncthreads();                              // every wave's records are written
    const uint32_t nev = s_evn;
    // with fewer chunks of events than waves (FUSE), the first waves run
    // them while the others flush the deposit: each wave waits only on its
    // own memory operations, so the events pass does not wait for the
    // flush's atomics to complete
    const uint32_t nch = FUSE ? (nev + 63u) >> 6 : 0u;
    const int quiet = nch < (uint32_t)kWavesPerTile ? (int)nch * 64 : 0;
    if (cur_g >= 0) flush(cur_g, quiet);
    if (tid == kBS - 1) d.evg[blockIdx.x] = nev;  // the events pass's count of this range
    if (FUSE) {
        // this workgroup's own events, in chunks of 64 over its waves:
        // the same pass as the events kernel's, on the records and the
        // tiles this workgroup has just written
        const EvPass ps{T, chunk, NT, (uint32_t)(T / kBirthsDiv), a.diag, a.eepf_inv_bin};
        for (uint32_t kc = (uint32_t)wid; kc < nch; kc += (uint32_t)kWavesPerTile) {
            uint4 rec, rq;
            const bool act = event_record(d, ps, (int)blockIdx.x, nev, kc, rec, rq);
            event_chunk(d, s_pref, NS, ps, act, rec, rq);
        }
    }
}

namespace {

// The collision of a candidate, in FP64: the energy (electrons: target at
// rest; ions: relative to a neutral drawn from the gas), the channel by the
// running sum of the tabulated frequencies against the second word of the
// first draw, then the kinematics of the channel.  Returns the channel (-1:
// null collision); `viol` says whether the summed frequency exceeded the
// bound, `born` whether an ionization filled the velocities of `bb` (the
// ejected electron and the new ion; the caller places them at the parent's
// position).
__device__ __forceinline__ int collide_particle(const SegConst& sc, const DisConst& dc, int s, uint32_t step,
                                                double& ux, double& uy, double& uz, uint32_t pid, Birth& bb,
                                                bool& viol, bool& born)
{
    const uint4 r = philox10(pid, step, ((uint32_t)s << 24), 0u, dc.key0, dc.key1);
    double speed, eps;
    double nvx = 0.0, nvy = 0.0, nvz = 0.0;
    if (!sc.ion_type) {
        const double v2 = ux * ux + uy * uy + uz * uz;
        speed = sqrt(v2);
        eps = sc.half_m_over_e_d * v2;
    } else {
        const uint4 r3 = philox10(pid, step, ((uint32_t)s << 24) | 3u, 0u, dc.key0, dc.key1);
        double g0, g1, g2, g3;
        box_muller_d(u01d(r3.x), u01d(r3.y), g0, g1);
        box_muller_d(u01d(r3.z), u01d(r3.w), g2, g3);
        nvx = sc.vt_gas * g0;
        nvy = sc.vt_gas * g1;
        nvz = sc.vt_gas * g2;
        const double gx = ux - nvx, gy = uy - nvy, gz = uz - nvz;
        const double g2s = gx * gx + gy * gy + gz * gz;
        speed = sqrt(g2s);
        eps = sc.half_m_over_e_d * g2s;
    }
    // channel: the first k whose running sum of n_g sigma_k g / nu_max passes
    // u1, one pass over the table row (the full sum checks the bound)
    const double u1 = u01d(r.y);
    double cum = 0.0;
    int ch = -1;
    {
        const double lx = (log(fmax(eps, 1e-300)) - sc.xs_ln0) * sc.xs_inv_dln;
        int i;
        double fr;
        if (!(lx > 0.0)) {
            i = 0;
            fr = 0.0;
        } else if (lx >= (double)(sc.xs_n - 1)) {
            i = sc.xs_n - 2;
            fr = 1.0;
        } else {
            i = (int)lx;
            if (i > sc.xs_n - 2) i = sc.xs_n - 2;
            fr = lx - (double)i;
        }
        const double* r0 = sc.xs + (size_t)i * sc.nch;
        const double* r1 = r0 + sc.nch;
        for (int k = 0; k < sc.nch; ++k) {
            const double v = r0[k] + fr * (r1[k] - r0[k]);
            cum += ((eps < sc.th[k]) ? 0.0 : v) * speed;
            if (ch < 0 && u1 < cum) ch = k;
        }
    }
    viol = cum > 1.0;
    born = false;
    if (ch < 0) return -1;
    const double cos_chi = 1.0 - 2.0 * u01d(r.z);
    const double u_phi = u01d(r.w);           // azimuth 2 pi u_phi
    const int kind = sc.kind[ch];
    if (!sc.ion_type) {
        const double inv = 1.0 / speed;
        const double dx_ = ux * inv, dy_ = uy * inv, dz_ = uz * inv;
        double ndx, ndy, ndz;
        scatter_dir_d(dx_, dy_, dz_, cos_chi, u_phi, ndx, ndy, ndz);
        double enew;
        if (kind == PIC_XS_ELASTIC) {
            enew = eps * (1.0 - sc.mr2 * (1.0 - cos_chi));
        } else if (kind == PIC_XS_EXCITATION) {
            enew = eps - sc.th[ch];
        } else {
            const uint4 r1 = philox10(pid, step, ((uint32_t)s << 24) | 1u, 0u, dc.key0, dc.key1);
            const uint4 r2 = philox10(pid, step, ((uint32_t)s << 24) | 2u, 0u, dc.key0, dc.key1);
            const double avail = eps - sc.th[ch];
            const double eej = u01d(r1.x) * avail;
            enew = avail - eej;
            double edx, edy, edz;
            scatter_dir_d(dx_, dy_, dz_, 1.0 - 2.0 * u01d(r1.y), u01d(r1.z), edx, edy, edz);
            const double vej = sqrt(sc.two_e_over_m * eej);
            double g0, g1, g2, g3;
            box_muller_d(u01d(r2.x), u01d(r2.y), g0, g1);
            box_muller_d(u01d(r2.z), u01d(r2.w), g2, g3);
            bb.vx = (float)(vej * edx);
            bb.vy = (float)(vej * edy);
            bb.vz = (float)(vej * edz);
            bb.ivx = (float)(sc.vt_gas * g0);
            bb.ivy = (float)(sc.vt_gas * g1);
            bb.ivz = (float)(sc.vt_gas * g2);
            born = true;
        }
        enew = fmax(enew, 0.0);
        const double vs = sqrt(sc.two_e_over_m * enew);
        ux = vs * ndx;
        uy = vs * ndy;
        uz = vs * ndz;
    } else if (kind == PIC_XS_ION_CX) {
        ux = nvx;
        uy = nvy;
        uz = nvz;
    } else {
        const double cmx = sc.m_frac * ux + sc.M_frac * nvx;
        const double cmy = sc.m_frac * uy + sc.M_frac * nvy;
        const double cmz = sc.m_frac * uz + sc.M_frac * nvz;
        const double st_ = sqrt(fmax(0.0, 1.0 - cos_chi * cos_chi));
        double sp_, cp_;
        sincospi(2.0 * u_phi, &sp_, &cp_);
        const double gg = sc.M_frac * speed;
        ux = cmx + gg * cos_chi;
        uy = cmy + gg * st_ * cp_;
        uz = cmz + gg * st_ * sp_;
    }
    return ch;
}

// The secondary electron of an ion absorbed at `wall`, in FP64: emitted with
// probability gamma (integer test on the draw), normal speed from the
// flux-weighted half-Maxwellian, tangential components Maxwellian, placed
// u v_n dt into the gap.  Returns 1 with `bb` filled when one is placed,
// -1 when one is emitted but lands beyond the gap, 0 when none is emitted.
__device__ __forceinline__ int secondary(const SegConst& sc, const DisConst& dc, int s, uint32_t step, int wall,
                                         uint32_t pid, Birth& bb)
{
    const uint4 r4 = philox10(pid, step, ((uint32_t)s << 24) | 4u, 0u, dc.key0, dc.key1);
    if (!(odd24(r4.x) < sc.see_k)) return 0;
    const uint4 r5 = philox10(pid, step, ((uint32_t)s << 24) | 5u, 0u, dc.key0, dc.key1);
    const int nc = dc.n_cells;
    const double vn = sc.vsee * sqrt(-2.0 * log(u01d(r4.y)));
    const double adv = u01d(r4.z) * vn * sc.dtdx_e;         // cells
    double g0, g1;
    box_muller_d(u01d(r5.x), u01d(r5.y), g0, g1);
    if (!(adv < (double)nc)) return -1;
    const double pos = wall == 0 ? adv : (double)nc - adv;   // cells from x = 0
    const double cf = floor(pos);
    int cell = (int)cf;
    float off = (float)(pos - cf);
    if (off >= 1.0f) {                   // the edge rule
        off -= 1.0f;
        cell += 1;
    }
    if (cell >= nc) {                    // within rounding of x = L: the last representable offset
        cell = nc - 1;
        off = 0x1.fffffep-1f;
    }
    if (cell < 0) return -1;
    bb.cell = cell;
    bb.off = off;
    bb.vx = (float)(wall == 0 ? vn : -vn);
    bb.vy = (float)(sc.vsee * g0);
    bb.vz = (float)(sc.vsee * g1);
    bb.ivx = bb.ivy = bb.ivz = 0.0f;
    return 1;
}

__device__ __forceinline__ uint32_t popc_ballot(bool p) { return (uint32_t)__popcll(__ballot(p)); }

}  // namespace

// This lane's event of chunk kc (events 64 kc .. 64 kc + 63) of the nev that
// push workgroup g recorded: its two record words; false past the list's end.
__device__ __forceinline__ bool event_record(const DevPtrs& d, const EvPass& ps, int g, uint32_t nev, uint32_t kc,
                                             uint4& rec, uint4& rq)
{
    const uint32_t e = (kc << 6) + (uint32_t)(threadIdx.x & 63);
    if (e >= nev) return false;
    const size_t ri = (size_t)g * ps.chunk_t * ps.T + e;
    rec = d.evr[ri];
    rq = d.evq[ri];
    return true;
}

// The events pass on one chunk: lanes with `act` hold an event's records.
__device__ __forceinline__ void event_chunk(const DevPtrs& d, const int32_t* s_pref, int NS, const EvPass& ps,
                                            bool act, uint4 rec, uint4 rq)
{
    const int S = d.S;
    const int lane = threadIdx.x & 63;
    bool hb = false, see = false, cand = false, viol = false, lost = false;
    int wall = 0, ch = -1, sg = -1;
    if (act) {
        const int32_t t = (int32_t)rq.w;
        const uint32_t word = rec.x;
        sg = (int)(word >> kEvSegShift);
        const int b = sg / S, s = sg - b * S;
        const DisConst& dc = d.disc[b];
        const SegConst& sc = d.segc[sg];
        const int32_t tin = t - s_pref[sg];
        const int io = d.segs[sg].parity;
        const uint32_t step = (uint32_t)d.diss[b].step;
        const int nc = dc.n_cells;
        const int periodic = dc.bc == PIC_BC_PERIODIC;
        const uint32_t key = word & kEvSlot;
        const int64_t slot = (int64_t)tin * ps.T + key;
        const uint32_t pid = rec.y;
        Birth bb;
        if (word & kEvSee) {
            see = true;
            wall = (word & kEvWall1) ? 1 : 0;
            const int r = secondary(sc, dc, s, step, wall, pid, bb);
            hb = r > 0;
            lost = r < 0;
        } else {
            double ux = __uint_as_float(rec.z), uy = __uint_as_float(rec.w), uz = __uint_as_float(rq.x);
            if (word & kEvRenew) {
                const uint4 r6 = philox10(pid, step, ((uint32_t)s << 24) | 6u, 0u, dc.key0, dc.key1);
                double g0, g1, g2, g3;
                box_muller_d(u01d(r6.x), u01d(r6.y), g0, g1);
                box_muller_d(u01d(r6.z), u01d(r6.w), g2, g3);
                ux = sc.drift0[0] + sc.vth0 * g0;
                uy = sc.drift0[1] + sc.vth0 * g1;
                uz = sc.drift0[2] + sc.vth0 * g2;
            }
            if (word & kEvCand) {
                cand = true;
                ch = collide_particle(sc, dc, s, step, ux, uy, uz, pid, bb, viol, hb);
            }
            // the position (the push's, in the record): for an ionization's
            // pair and the diagnostics
            const int c = (int)rq.y;
            const float f = __uint_as_float(rq.z);
            if (hb) {
                bb.cell = c;
                bb.off = f;
            }
            const float fx = (float)ux, fy = (float)uy, fz = (float)uz;
            sc.vx[io][slot] = fx;
            sc.vy[io][slot] = fy;
            sc.vz[io][slot] = fz;
            if (ps.diag) {
                unsigned long long* fh = d.macc + (size_t)sg * 2 * d.nodes_max;
                moment_diag(sc.mscale1, sc.mscale2, fh, fh + d.nodes_max, c, f, fx, nc, periodic);
                if (s == 0)
                    electron_diag(sc.half_m_over_e, dc.bulk_lo, dc.bulk_hi, ps.eepf_inv_bin,
                                  d.eacc + (size_t)b * d.nodes_max,
                                  d.eepf + (size_t)b * 2 * kEepfBins, c, f, fx, fy, fz, nc, periodic);
            }
        }
        if (hb) {
            const uint32_t pos = atomicAdd(reinterpret_cast<uint32_t*>(&d.bcnt[t]), 1u);
            if (pos < ps.bpt) {
                bb.key = key;
                d.births[(size_t)t * ps.bpt + pos] = bb;
                unsigned long long* acc_e = d.acc + ((size_t)b * S + 0) * kRep * d.nodes_max;
                global_deposit(acc_e, bb.cell, bb.off, nc, periodic);
                if (!see && S > 1)          // no ions in a swarm
                    global_deposit(d.acc + ((size_t)b * S + 1) * kRep * d.nodes_max, bb.cell, bb.off, nc,
                                   periodic);
                if (ps.diag) {
                    // the births' velocity moments and the electron's
                    // energy, with the particles of the step
                    const SegConst& se = d.segc[b * S + 0];
                    unsigned long long* fe = d.macc + (size_t)(b * S + 0) * 2 * d.nodes_max;
                    moment_diag(se.mscale1, se.mscale2, fe, fe + d.nodes_max, bb.cell, bb.off, bb.vx, nc,
                                periodic);
                    electron_diag(se.half_m_over_e, dc.bulk_lo, dc.bulk_hi, ps.eepf_inv_bin,
                                  d.eacc + (size_t)b * d.nodes_max, d.eepf + (size_t)b * 2 * kEepfBins,
                                  bb.cell, bb.off, bb.vx, bb.vy, bb.vz, nc, periodic);
                    if (!see && S > 1) {
                        const SegConst& si = d.segc[b * S + 1];
                        unsigned long long* fi = d.macc + (size_t)(b * S + 1) * 2 * d.nodes_max;
                        moment_diag(si.mscale1, si.mscale2, fi, fi + d.nodes_max, bb.cell, bb.off, bb.ivx, nc,
                                    periodic);
                    }
                }
                atomicAdd(reinterpret_cast<unsigned long long*>(&d.segs[sg].staged), 1ull);
            } else {
                hb = false;
                lost = true;
                atomicOr(&d.diss[b].flags, kFlagCapacity);
            }
        }
    }
    // counters of the chunk, one segment at a time (a chunk spans more
    // than one only at a segment's end): lane i holds counter i
    uint64_t todo = __ballot(act);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lsg = __shfl(sg, leader, 64);
        const bool mine = act && sg == lsg;
        uint32_t cnt_lane = 0u;
        auto count = [&](int i, bool p) {
            const uint32_t v = popc_ballot(mine && p);
            cnt_lane += lane == i ? v : 0u;
        };
        count(C_CAND, cand);
        count(C_NULL, cand && ch < 0);
        count(C_VIOL, viol);
        const int nch = d.segc[lsg].nch;
        for (int k = 0; k < nch; ++k) count(C_COLL + k, ch == k);
        count(C_SEE0, hb && see && wall == 0);
        count(C_SEE1, hb && see && wall == 1);
        count(C_DROP, lost);
        if (lane < C_N && cnt_lane)
            atomicAdd(&d.cnt[((size_t)lsg * kRep) * C_N + lane], (unsigned long long)cnt_lane);
        todo &= ~__ballot(mine);
    }
}

// The events of a step, after the push: chunks of 64 consecutive events of
// one push workgroup's range (in unit order: tiles, waves, slots), fully
// packed but for the last of each range, strided over all the waves of the
// grid.  Each lane one event: the renewal
// (a fresh velocity from the species' initial distribution, call 6), the
// collision of a candidate, or the secondary-emission test of an absorbed
// ion, all in FP64, with the new velocity rounded to binary32 once and
// written to the particle's slot, and the diagnostics of the particle's
// final velocity.  A birth (ionization pair, secondary electron) claims a
// slot of its tile's staging area with an atomic and carries its parent's
// slot, by which the finalize orders the tile's births; its charge goes
// straight into the discharge's fixed-point sums.  Counters come from
// ballots, per segment of the chunk.
template <int BS>
__global__ __launch_bounds__(BS) void events_kernel(EvArgs a)
{
    const DevPtrs& d = a.d;
    const int NS = d.B * d.S;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int kW = BS / 64;
    __shared__ int32_t s_pref[kMaxSeg + 1];
    __shared__ uint32_t s_cp[kMaxPushGrid + 1];   // chunks of the push workgroups before each
    __shared__ uint32_t s_ne[kMaxPushGrid];       // events of each push workgroup
    __shared__ uint32_t s_w[kW];
    tile_prefix(d, a.T, s_pref);
    const int G = a.push_grid;
    uint32_t run = 0;
    for (int r = 0; r < G; r += BS) {
        const int g = r + tid;
        const uint32_t ne = g < G ? d.evg[g] : 0u;
        const uint32_t c = (ne + 63u) >> 6;
        if (g < G) s_ne[g] = ne;
        const uint32_t incl = wave_incl_scan_u32(c);
        if (lane == 63) s_w[wid] = incl;
        __syncthreads();
        uint32_t before = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < kW; ++k) {
            const uint32_t v = s_w[k];
            if (k < wid) before += v;
            tot += v;
        }
        if (g < G) s_cp[g] = run + before + incl - c;
        run += tot;
        __syncthreads();
    }
    if (tid == 0) s_cp[G] = run;
    __syncthreads();
    const int32_t NT = s_pref[NS];
    const int32_t chunk_t = (NT + G - 1) / G;     // the push workgroups' tile ranges
    const uint32_t bpt = (uint32_t)a.births_per_tile;
    const uint32_t nchunk = s_cp[G];
    const uint32_t stride = gridDim.x * kW;

    const EvPass e{a.T, chunk_t, NT, bpt, a.diag, a.eepf_inv_bin};
    // the records of chunk ck, for the lanes that hold one; the push
    // workgroup of chunk ck is the last g with s_cp[g] <= ck
    auto records = [&](uint32_t ck, uint4& rec, uint4& rq) -> bool {
        int glo = 0, ghi = G;
        while (ghi - glo > 1) {
            const int mid = (glo + ghi) >> 1;
            if (s_cp[mid] <= ck) glo = mid; else ghi = mid;
        }
        return event_record(d, e, glo, s_ne[glo], ck - s_cp[glo], rec, rq);
    };
    // each wave's next chunk's records are loaded before it works on the
    // current one, so that their latency overlaps the current chunk's loads
    uint32_t ck = blockIdx.x * kW + wid;
    uint4 rec = make_uint4(0u, 0u, 0u, 0u), rq = rec;
    bool act = ck < nchunk && records(ck, rec, rq);
    while (ck < nchunk) {
        const uint32_t nx = ck + stride;
        uint4 rec_n = make_uint4(0u, 0u, 0u, 0u), rq_n = rec_n;
        const bool act_n = nx < nchunk && records(nx, rec_n, rq_n);
        event_chunk(d, s_pref, NS, e, act, rec, rq);
        rec = rec_n;
        rq = rq_n;
        act = act_n;
        ck = nx;
    }
}

#define PIC_KERNELS(X)        \
    X(1, 256, false, false)   \
    X(2, 256, false, false)   \
    X(4, 256, false, false)   \
    X(8, 256, false, false)   \
    X(4, 512, false, false)   \
    X(4, 1024, false, false)  \
    X(1, 256, true, false)    \
    X(2, 256, true, false)    \
    X(4, 256, true, false)    \
    X(4, 512, true, false)    \
    X(4, 1024, true, false)   \
    X(8, 256, true, false)    \
    X(8, 512, true, false)    \
    X(1, 256, true, true)     \
    X(2, 256, true, true)     \
    X(4, 256, true, true)

#define PIC_INST(P, B, G, F) template __global__ void push_kernel<P, B, G, F>(PushArgs);
PIC_KERNELS(PIC_INST)
#undef PIC_INST

size_t push_lds_bytes(int n_nodes, int n_cells, int diag)
{
    size_t b = (size_t)n_nodes * 8;
    if (diag) b += (size_t)n_nodes * 8 * 3 + kEepfBins * 4;
    b = (b + 15) & ~(size_t)15;
    b += (size_t)n_cells * 8;
    return b;
}

// nearest instantiated shape (1024 threads: four particles per thread; 512:
// four, or eight in the general kernel; 256: one to eight)
void push_shape(int& ppt, int& threads, bool general)
{
    if (threads >= 1024) {
        threads = 1024;
        ppt = 4;
    } else if (threads >= 512) {
        threads = 512;
        ppt = (general && ppt >= 8) ? 8 : 4;
    } else {
        threads = 256;
        ppt = ppt >= 8 ? 8 : (ppt >= 4 ? 4 : (ppt >= 2 ? 2 : 1));
    }
}

bool push_fusable(int ppt, int threads, bool general) { return general && threads == 256 && ppt <= 4; }

hipError_t launch_push(const PushArgs& a, int ppt, int threads, bool general, bool fuse, int64_t grid,
                       hipStream_t st)
{
    const size_t lds = push_lds_bytes(a.nodes_max_dyn, a.cells_max_dyn, a.diag);
    const dim3 g((unsigned)grid);
#define PIC_LAUNCH(P, B, G, F)                                                           \
    if (ppt == P && threads == B && general == G && fuse == F) {                         \
        hipLaunchKernelGGL((push_kernel<P, B, G, F>), g, dim3(B), lds, st, a);          \
        return hipGetLastError();                                                        \
    }
    PIC_KERNELS(PIC_LAUNCH)
#undef PIC_LAUNCH
    return hipErrorInvalidValue;
}

int push_occupancy(int ppt, int threads, bool general, bool fuse, size_t lds)
{
    int nb = 0;
#define PIC_OCC(P, B, G, F)                                                                         \
    if (ppt == P && threads == B && general == G && fuse == F) {                                    \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(                                           \
                &nb, reinterpret_cast<const void*>(push_kernel<P, B, G, F>), B, lds) != hipSuccess)  \
            nb = 0;                                                                                 \
    }
    PIC_KERNELS(PIC_OCC)
#undef PIC_OCC
    return nb > 0 ? nb : 1;
}

template __global__ void events_kernel<kEvThreads>(EvArgs);

hipError_t launch_events(const EvArgs& a, int64_t grid, hipStream_t st)
{
    hipLaunchKernelGGL((events_kernel<kEvThreads>), dim3((unsigned)grid), dim3(kEvThreads), 0, st, a);
    return hipGetLastError();
}

int events_occupancy()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(events_kernel<kEvThreads>),
                                                     kEvThreads, 0) != hipSuccess)
        nb = 0;
    return nb > 0 ? nb : 1;
}

}  // namespace pic
