// Host side of the C ABI declared in include/pic.h: validation, device
// allocation, the per-species constants of the push, the collision tables and
// their frequency bound, kernel launches, and diagnostics readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "pic.h"
#include "pic_internal.h"
#include "pic_kernels.h"

using namespace pic;

namespace {

constexpr double kBoltzmann = 1.380649e-23;
constexpr int kTileMax = 4096;     // largest tile (1024 threads x 4): capacities are padded to it

struct Table {
    int32_t kind;
    double th;
    std::vector<double> e, s;
};

struct SegHost {
    std::vector<Table> tabs;
    double numax = 0.0;
    uint32_t t32 = 0;
    void* xs_dev = nullptr;
};

}  // namespace

struct pic_ctx {
    hipStream_t stream = nullptr;
    pic_allocator alloc{};
    bool has_alloc = false;
    int B = 0, S = 0;
    std::vector<pic_config> cfg;
    std::vector<SegConst> segc;
    std::vector<SegHost> segh;
    std::vector<DisConst> disc;
    DevPtrs d{};
    std::vector<void*> blocks;
    int ppt = 4;                          // particles per thread
    int threads = 1024;                   // threads per workgroup (streaming kernels)
    int n_cu = 256;
    int device = 0;                       // the GPU current at pic_init
    int sort_every = 0;
    int64_t steps_since_sort = 0;
    int compact_every = 16;              // steps between compactions of the holes
    int events_in_push = 0;              // 256-thread general pushes do their own events
    int64_t steps_since_compact = 0;
    int64_t compact_tiles = 0;           // grid of the compaction passes
    int diag = 0;
    double eepf_emax = 64.0;
    double wedf_emax[PIC_MAX_SPECIES] = {64.0, 1024.0, 1024.0, 1024.0};   // wall impact-energy ranges (eV)
    double* poisson_scratch = nullptr;   // rho, phi, e: 3 * nodes_max
    void* sort_scratch = nullptr;
    size_t sort_scratch_bytes = 0;
    int64_t sort_tiles = 0;
    std::vector<int64_t> grid_cap;       // per species: sum over discharges of padded capacity
    // live timing of launches (pic_profile)
    int prof = 0;
    std::vector<hipEvent_t> ev;           // pool, reused
    std::vector<std::pair<int, int>> pending;  // (kind, first event index); kind = species or -1 finalize
    size_t ev_used = 0;
    double push_ms = 0.0, push_n = 0.0;
    double fin_ms = 0.0, fin_n = 0.0;
    double ev_ms = 0.0, ev_n = 0.0;
    // replay of a captured chunk of steps
    int use_graph = 1;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    int g_steps = 0;
    int64_t graph_replays = 0, graph_steps = 0;   // replays of captured chunks since pic_init, and their steps
    uint64_t g_key = 0;
};

namespace {

void* dev_alloc(pic_ctx* c, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    void* p = nullptr;
    if (c->has_alloc) {
        p = c->alloc.alloc(bytes, c->alloc.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) c->blocks.push_back(p);
    return p;
}

void dev_release(pic_ctx* c, void* p)
{
    if (!p) return;
    auto it = std::find(c->blocks.begin(), c->blocks.end(), p);
    if (it != c->blocks.end()) c->blocks.erase(it);
    if (c->has_alloc) c->alloc.free(p, c->alloc.user);
    else (void)hipFree(p);
}

bool valid_species(const pic_species_cfg& s)
{
    return s.mass > 0.0 && std::isfinite(s.mass) && std::isfinite(s.charge) && s.weight > 0.0 &&
           s.capacity >= s.n_init && s.n_init >= 0 && s.capacity <= (int64_t(1) << 31) &&
           s.load >= PIC_LOAD_STRATIFIED && s.load <= PIC_LOAD_NONE && s.vth >= 0.0;
}

pic_status check_cfg(const pic_config& c)
{
    if (c.n_cells < 2 || c.n_cells > kMaxCells) return PIC_EINVAL;
    if (c.bc == PIC_BC_DIRICHLET && c.n_cells + 1 > kFinThreads * kNodesPerThread) return PIC_EINVAL;
    if (c.bc != PIC_BC_PERIODIC && c.bc != PIC_BC_DIRICHLET) return PIC_EINVAL;
    if (!(c.length > 0.0) || !(c.dt > 0.0) || !(c.eps0 > 0.0) || !(c.e_unit > 0.0)) return PIC_EINVAL;
    if (c.n_species < 1 || c.n_species > PIC_MAX_SPECIES) return PIC_EINVAL;
    if (c.see_gamma < 0.0 || c.see_gamma > 1.0) return PIC_EINVAL;
    if (!(c.renew_lz >= 0.0) || !std::isfinite(c.renew_lz)) return PIC_EINVAL;
    if (c.drive < PIC_DRIVE_VOLTAGE || c.drive > PIC_DRIVE_CURRENT) return PIC_EINVAL;
    if (c.bc == PIC_BC_PERIODIC && c.drive != PIC_DRIVE_VOLTAGE) return PIC_EINVAL;
    if (c.waveform != PIC_WAVE_SINE && c.waveform != PIC_WAVE_TWO_HARMONIC) return PIC_EINVAL;
    if (!(c.cap >= 0.0) || !std::isfinite(c.cap) || !std::isfinite(c.j_amp)) return PIC_EINVAL;
    for (int s = 0; s < c.n_species; ++s)
        if (!valid_species(c.species[s])) return PIC_EINVAL;
    return PIC_OK;
}

int64_t pad_cap(int64_t cap) { return std::max<int64_t>(kTileMax, (cap + kTileMax - 1) / kTileMax * kTileMax); }

pic_status hip_st(hipError_t e) { return e == hipSuccess ? PIC_OK : PIC_EHIP; }

// sigma(eps) of one table: linear in ln(eps), end values outside, zero below threshold
double sigma_of(const Table& t, double eps)
{
    if (eps < t.th) return 0.0;
    const size_t n = t.e.size();
    if (eps <= t.e[0]) return t.s[0];
    if (eps >= t.e[n - 1]) return t.s[n - 1];
    size_t lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        const size_t mid = (lo + hi) / 2;
        if (t.e[mid] <= eps) lo = mid; else hi = mid;
    }
    const double u = (std::log(eps) - std::log(t.e[lo])) / (std::log(t.e[hi]) - std::log(t.e[lo]));
    return t.s[lo] + u * (t.s[hi] - t.s[lo]);
}

bool electron_kind(int k) { return k == PIC_XS_ELASTIC || k == PIC_XS_EXCITATION || k == PIC_XS_IONIZATION; }

// Upper bound of the collision frequency and the integer candidate threshold.
// Electron-type: 1.05 x max over a log-uniform grid ten times finer than the
// longest table of n_g sum_k sigma_k(eps) sqrt(2 e eps / m).  Ion-type:
// n_g max(sum_k sigma_k) g_max, g_max = sqrt(2 e eps_top / m) + 6 sqrt(k T_g / M).
void bound(const pic_config& c, int s, SegHost& h)
{
    const auto& T = h.tabs;
    double elo = T[0].e.front(), ehi = T[0].e.back();
    size_t nmax = 0;
    for (const auto& t : T) {
        elo = std::min(elo, t.e.front());
        ehi = std::max(ehi, t.e.back());
        nmax = std::max(nmax, t.e.size());
    }
    const int m = 10 * (int)nmax;
    const double lelo = std::log(elo), lehi = std::log(ehi);
    const double mass = c.species[s].mass, ng = c.gas_density;
    const bool ion = !electron_kind(T[0].kind);
    double best = 0.0;
    for (int j = 0; j < m; ++j) {
        const double eps = std::exp(lelo + (double)j * (lehi - lelo) / (double)(m - 1));
        double sig = 0.0;
        for (const auto& t : T) sig += sigma_of(t, eps);
        const double val = ion ? sig : ng * sig * std::sqrt(2.0 * c.e_unit * eps / mass);
        if (val > best) best = val;
    }
    double numax;
    if (ion) {
        const double gmax = std::sqrt(2.0 * c.e_unit * ehi / mass) +
                            6.0 * std::sqrt(kBoltzmann * c.gas_temp / c.gas_mass);
        numax = ng * best * gmax;
    } else {
        numax = 1.05 * best;
    }
    const double pnull = 1.0 - std::exp(-numax * c.dt);
    double t = std::floor(pnull * 4294967296.0);
    if (t > 4294967295.0) t = 4294967295.0;
    h.numax = numax;
    h.t32 = (uint32_t)t;
}

// velocity scale of the fixed-point moments: the speed of a 50 eV particle
// of the species (|vx| up to ~2^15 of it stays exact in the int64 sums)
constexpr double kMomentScale = 16777216.0;   // 2^24
double moment_vref(const pic_config& c, int s) { return std::sqrt(100.0 * c.e_unit / c.species[s].mass); }

void fill_push_consts(const pic_config& c, int s, SegConst& sc)
{
    const pic_species_cfg& sp = c.species[s];
    const double dx = c.length / c.n_cells;
    const double qm = sp.charge / sp.mass;
    sc.qm = qm;
    sc.qmh = (float)(0.5 * qm * c.dt);
    double t[3], t2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        t[k] = 0.5 * qm * c.b_ext[k] * c.dt;
        t2 += t[k] * t[k];
    }
    for (int k = 0; k < 3; ++k) {
        sc.tv[k] = (float)t[k];
        sc.sv[k] = (float)(2.0 * t[k] / (1.0 + t2));
        sc.eext[k] = (float)c.e_ext[k];
    }
    sc.dtdx = (float)(c.dt / dx);
    sc.mw_half = 0.5 * sp.mass * sp.weight;
    sc.q = sp.charge;
    sc.w = sp.weight;
    sc.mass = (float)sp.mass;
    sc.compacts = c.bc == PIC_BC_DIRICHLET ? 1 : 0;
    sc.half_m_over_e = (float)(0.5 * sp.mass / c.e_unit);
    sc.half_m_over_e_d = 0.5 * sp.mass / c.e_unit;
    sc.two_e_over_m = 2.0 * c.e_unit / sp.mass;
    sc.mscale1 = (float)(kMomentScale / moment_vref(c, s));
    sc.mscale2 = (float)(kMomentScale / (moment_vref(c, s) * moment_vref(c, s)));
    sc.wedf_inv_bin = (float)(kEepfBins / (s == 0 ? 64.0 : 1024.0));
    sc.renew_lz = c.renew_lz;
    sc.dt_d = c.dt;
    sc.vth0 = sp.vth;
    for (int k = 0; k < 3; ++k) sc.drift0[k] = sp.drift[k];
    sc.emits = (s >= 1 && sp.charge > 0.0 && c.see_gamma > 0.0 && c.bc == PIC_BC_DIRICHLET) ? 1 : 0;
    sc.see_k = (uint32_t)std::min(16777217.0, std::ceil(c.see_gamma * 16777216.0));
    sc.vsee = std::sqrt(c.see_temp * c.e_unit / c.species[0].mass);
    sc.dtdx_e = c.dt / dx;
}

// Collision constants of a segment from its host tables: the frequency bound,
// and the table n_g sigma_k / nu_max on a uniform ln(eps) grid (the input grid
// itself when every process shares one log-uniform grid, else 4096 points).
pic_status build_xs(pic_ctx* ctx, int b, int s)
{
    const pic_config& c = ctx->cfg[b];
    SegHost& h = ctx->segh[b * ctx->S + s];
    SegConst& sc = ctx->segc[b * ctx->S + s];
    const int nch = (int)h.tabs.size();
    bound(c, s, h);
    bool shared = true;
    const auto& e0 = h.tabs[0].e;
    for (const auto& t : h.tabs)
        if (t.e != e0) shared = false;
    if (shared && e0.size() >= 2) {
        const double hstep = (std::log(e0.back()) - std::log(e0.front())) / (double)(e0.size() - 1);
        for (size_t i = 0; i + 1 < e0.size(); ++i) {
            const double d = std::log(e0[i + 1]) - std::log(e0[i]);
            if (std::fabs(d - hstep) > 1e-9 * hstep) {
                shared = false;
                break;
            }
        }
    }
    double elo = e0.front(), ehi = e0.back();
    for (const auto& t : h.tabs) {
        elo = std::min(elo, t.e.front());
        ehi = std::max(ehi, t.e.back());
    }
    const int n = shared ? (int)e0.size() : 4096;
    const double l0 = std::log(elo), l1 = std::log(ehi);
    std::vector<double> xs((size_t)n * nch);
    const double scale = c.gas_density / h.numax;
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < nch; ++k) {
            const Table& t = h.tabs[k];
            double sig;
            if (shared) {
                sig = t.s[i];
            } else {
                const double eps = std::exp(l0 + (l1 - l0) * (double)i / (double)(n - 1));
                const double keep_th = t.th;
                Table tt = t;
                tt.th = 0.0;              // threshold applied in the kernel
                sig = sigma_of(tt, eps);
                (void)keep_th;
            }
            xs[(size_t)i * nch + k] = sig * scale;
        }
    }
    void* p = dev_alloc(ctx, xs.size() * sizeof(double));
    if (!p) return PIC_ENOMEM;
    if (hipMemcpy(p, xs.data(), xs.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return PIC_EHIP;
    if (h.xs_dev) dev_release(ctx, h.xs_dev);
    h.xs_dev = p;
    sc.xs = (const double*)p;
    sc.xs_n = n;
    sc.xs_ln0 = l0;
    sc.xs_inv_dln = (double)(n - 1) / (l1 - l0);
    sc.nch = nch;
    sc.ion_type = electron_kind(h.tabs[0].kind) ? 0 : 1;
    sc.t32 = h.t32;
    for (int k = 0; k < nch; ++k) {
        sc.kind[k] = h.tabs[k].kind;
        sc.th[k] = h.tabs[k].th;
    }
    const double m = c.species[s].mass, M = c.gas_mass;
    sc.mr2 = 2.0 * m / M;
    sc.vt_gas = std::sqrt(kBoltzmann * c.gas_temp / M);
    sc.m_frac = m / (m + M);
    sc.M_frac = M / (m + M);
    return PIC_OK;
}

pic_status upload_segc(pic_ctx* ctx, int idx)
{
    return hip_st(hipMemcpy(ctx->d.segc + idx, &ctx->segc[idx], sizeof(SegConst), hipMemcpyHostToDevice));
}

pic_status flags_status(uint32_t f)
{
    if (f & kFlagStall) return PIC_ESTALL;
    if (f & kFlagCapacity) return PIC_ECAPACITY;
    if (f & (kFlagNumeric | kFlagCell)) return PIC_ENUMERIC;
    return PIC_OK;
}

int64_t max_count_of(pic_ctx* ctx, int only_b)
{
    int64_t m = 0;
    for (int b = 0; b < ctx->B; ++b) {
        if (only_b >= 0 && b != only_b) continue;
        for (int s = 0; s < ctx->S; ++s) m = std::max(m, ctx->segc[b * ctx->S + s].cap);
    }
    return m;
}

// event pair around a launch when profiling
int prof_begin(pic_ctx* c)
{
    if (!c->prof) return -1;
    if (c->ev_used + 2 > c->ev.size()) {
        for (int k = 0; k < 64; ++k) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            c->ev.push_back(e);
        }
    }
    const int i = (int)c->ev_used;
    c->ev_used += 2;
    (void)hipEventRecord(c->ev[i], c->stream);
    return i;
}

void prof_end(pic_ctx* c, int i, int kind)
{
    if (i < 0) return;
    (void)hipEventRecord(c->ev[i + 1], c->stream);
    c->pending.emplace_back(kind, i);
}

// fold finished event pairs into the sums
void prof_collect(pic_ctx* c)
{
    if (c->pending.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& pr : c->pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->ev[pr.second], c->ev[pr.second + 1]) != hipSuccess) continue;
        if (pr.first < 0) {
            c->fin_ms += ms;
            c->fin_n += 1.0;
        } else if (pr.first == 1) {
            c->ev_ms += ms;
            c->ev_n += 1.0;
        } else {
            c->push_ms += ms;
            c->push_n += 1.0;
        }
    }
    c->pending.clear();
    c->ev_used = 0;
}

pic_status solve_after_deposit(pic_ctx* ctx, int only_b)
{
    if (launch_deposit(ctx->d, only_b, max_count_of(ctx, only_b), ctx->stream) != hipSuccess) return PIC_EHIP;
    FinArgs fa{};
    fa.d = ctx->d;
    fa.mode = kFinSolve;
    fa.only_b = only_b;
    if (launch_finalize(fa, ctx->stream) != hipSuccess) return PIC_EHIP;
    return PIC_OK;
}

}  // namespace

namespace {
void drop_graph(pic_ctx* ctx);
}

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free calls: one array per GPU, never freed.
// Its name is a host-side stand-in in host code; the device address of each
// GPU's copy is resolved once, with that GPU current, and kept here.
static __device__ __align__(256) unsigned char scratch[PIC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

pic_status noalloc_scratch_init(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return PIC_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return PIC_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PIC_EHIP;
    g_scratch_ptr[dev] = ptr;
    return PIC_OK;
}

void* noalloc_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

const char* pic_strerror(pic_status s)
{
    switch (s) {
        case PIC_OK: return "ok";
        case PIC_EINVAL: return "invalid argument";
        case PIC_ENOMEM: return "out of memory";
        case PIC_EHIP: return "HIP runtime error";
        case PIC_ECAPACITY: return "particle capacity exceeded";
        case PIC_ENUMERIC: return "non-finite or out-of-range particle state";
        case PIC_ESTATE: return "invalid state";
        case PIC_ESTALL: return "reserved status";
        case PIC_ESCRATCH: return "work larger than the fixed scratch of an allocation-free call";
        default: return "unknown status";
    }
}

void pic_free(pic_ctx* ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
    drop_graph(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    std::vector<void*> bl = ctx->blocks;
    for (void* p : bl) dev_release(ctx, p);
    delete ctx;
}

pic_status pic_init(const pic_config* cfg, int32_t n_batch, const pic_allocator* alloc, void* hip_stream,
                    pic_ctx** out)
{
    if (!cfg || !out || n_batch < 1 || n_batch > PIC_MAX_BATCH) return PIC_EINVAL;
    for (int b = 0; b < n_batch; ++b) {
        if (check_cfg(cfg[b]) != PIC_OK) return PIC_EINVAL;
        if (cfg[b].n_species != cfg[0].n_species) return PIC_EINVAL;
    }
    pic_ctx* ctx = new (std::nothrow) pic_ctx();
    if (!ctx) return PIC_ENOMEM;
    ctx->stream = (hipStream_t)hip_stream;
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            ctx->n_cu = prop.multiProcessorCount;
        ctx->device = dev;
        if (noalloc_scratch_init(dev) != PIC_OK) {
            delete ctx;
            return PIC_EHIP;
        }
    }
    if (alloc && alloc->alloc && alloc->free) {
        ctx->alloc = *alloc;
        ctx->has_alloc = true;
    }
    const int B = n_batch, S = cfg[0].n_species;
    ctx->B = B;
    ctx->S = S;
    ctx->cfg.assign(cfg, cfg + B);
    ctx->segc.assign((size_t)B * S, SegConst{});
    ctx->segh.assign((size_t)B * S, SegHost{});
    ctx->disc.assign(B, DisConst{});
    DevPtrs& d = ctx->d;
    d.B = B;
    d.S = S;
    int nodes_max = 0, cells_max = 0;
    for (int b = 0; b < B; ++b) {
        nodes_max = std::max(nodes_max, cfg[b].bc == PIC_BC_PERIODIC ? cfg[b].n_cells : cfg[b].n_cells + 1);
        cells_max = std::max(cells_max, cfg[b].n_cells);
    }
    d.nodes_max = nodes_max;
    d.cells_max = cells_max;
    ctx->grid_cap.assign(S, 0);
    pic_status rc = PIC_OK;
    auto A = [&](size_t bytes) -> void* {
        void* p = dev_alloc(ctx, bytes);
        if (!p) rc = PIC_ENOMEM;
        return p;
    };
    // particle storage
    for (int b = 0; b < B && rc == PIC_OK; ++b) {
        const pic_config& c = cfg[b];
        DisConst& dc = ctx->disc[b];
        dc.n_cells = c.n_cells;
        dc.n_nodes = c.bc == PIC_BC_PERIODIC ? c.n_cells : c.n_cells + 1;
        dc.bc = c.bc;
        dc.field_solve = c.field_solve ? 1 : 0;
        dc.dx = c.length / c.n_cells;
        dc.dt = c.dt;
        dc.L = c.length;
        dc.eps0 = c.eps0;
        dc.rho_bg = c.rho_bg;
        dc.v_amp = c.v_amp;
        dc.v_freq = c.v_freq;
        dc.v_phase = c.v_phase;
        for (int k = 0; k < 3; ++k) {
            dc.e_ext[k] = c.e_ext[k];
            dc.b_ext[k] = c.b_ext[k];
        }
        dc.c2 = dc.dx * dc.dx / c.eps0;
        dc.inv_2dx = 1.0 / (2.0 * dc.dx);
        dc.drive = c.drive;
        dc.waveform = c.waveform;
        dc.cap = c.cap;
        dc.j_amp = c.j_amp;
        for (int s = 0; s < c.n_species; ++s) dc.qw[s] = c.species[s].charge * c.species[s].weight;
        // bulk electron energy distribution: the middle tenth of a bounded
        // gap, every cell when periodic
        if (c.bc == PIC_BC_PERIODIC) {
            dc.bulk_lo = 0;
            dc.bulk_hi = c.n_cells;
        } else {
            dc.bulk_lo = (int)std::floor(0.45 * c.n_cells);
            dc.bulk_hi = std::max(dc.bulk_lo + 1, (int)std::ceil(0.55 * c.n_cells));
        }
        dc.inv_dx = 1.0 / dc.dx;
        dc.wall_coef = dc.dx / (2.0 * c.eps0);
        for (int s = 0; s < S; ++s) {
            dc.dens_coef[s] = c.species[s].weight / dc.dx / kDepScale;
            dc.q[s] = c.species[s].charge;
            dc.mass[s] = c.species[s].mass;
            dc.flux_coef[s] = c.species[s].weight / dc.dx / (kMomentScale / moment_vref(c, s));
            dc.mom_coef[s] = c.species[s].weight / dc.dx / (kMomentScale / (moment_vref(c, s) * moment_vref(c, s)));
        }
        dc.key0 = (uint32_t)(c.seed & 0xffffffffu);
        dc.key1 = (uint32_t)(c.seed >> 32);
        for (int s = 0; s < S && rc == PIC_OK; ++s) {
            SegConst& sc = ctx->segc[b * S + s];
            const int64_t cap = pad_cap(c.species[s].capacity);
            sc.cap = c.species[s].capacity;
            ctx->grid_cap[s] += cap;
            for (int k = 0; k < 2; ++k) {        // the compaction and the sort write the other copy
                sc.cell[k] = (int32_t*)A(cap * 4);
                sc.off[k] = (float*)A(cap * 4);
                sc.vx[k] = (float*)A(cap * 4);
                sc.vy[k] = (float*)A(cap * 4);
                sc.vz[k] = (float*)A(cap * 4);
                sc.id[k] = (uint32_t*)A(cap * 4);
                sc.z[k] = c.renew_lz > 0.0 ? (double*)A(cap * 8) : nullptr;
            }
            fill_push_consts(c, s, sc);
        }
    }
    ctx->compact_tiles = 0;
    for (int g = 0; g < B * S; ++g) ctx->compact_tiles += compact_tiles_for(pad_cap(ctx->segc[g].cap));
    // tiles are numbered over every segment of the context
    int64_t tiles_max = (int64_t)B * S;
    for (int s = 0; s < S; ++s) tiles_max += ctx->grid_cap[s] / kTileMin;
    if (tiles_max > kMaxTiles) rc = PIC_EINVAL;
    d.tiles_max = tiles_max;
    if (rc == PIC_OK) {
        d.segc = (SegConst*)A(sizeof(SegConst) * B * S);
        d.segs = (SegState*)A(sizeof(SegState) * B * S);
        d.disc = (DisConst*)A(sizeof(DisConst) * B);
        d.diss = (DisState*)A(sizeof(DisState) * B);
        d.acc = (unsigned long long*)A(8ull * B * S * kRep * nodes_max);
        d.cnt = (unsigned long long*)A(8ull * B * S * kRep * C_N);
        d.eacc = (unsigned long long*)A(8ull * B * nodes_max);
        d.macc = (unsigned long long*)A(8ull * B * S * 2 * nodes_max);
        d.pavg = (double*)A(8ull * B * S * kPow * nodes_max);
        d.gprev = (double*)A(8ull * B * S * nodes_max);
        d.ptmp = (double*)A(8ull * B * 2 * nodes_max);
        d.wen = (unsigned long long*)A(8ull * B * S * 2);
        d.rho = (double*)A(8ull * B * nodes_max);
        d.phi = (double*)A(8ull * B * nodes_max);
        d.ef = (double*)A(8ull * B * nodes_max);
        d.dens = (double*)A(8ull * B * S * nodes_max);
        d.epair = (float2*)A(8ull * B * cells_max);
        d.avg = (double*)A(8ull * B * (S + 2) * nodes_max);
        d.eepf = (unsigned long long*)A(8ull * B * 2 * kEepfBins);
        d.wedf = (unsigned long long*)A(8ull * B * S * 2 * kEepfBins);
        d.wring = (double*)A(8ull * B * kWindowRing * (1 + (size_t)(S + 2) * nodes_max));
        d.births = (Birth*)A(sizeof(Birth) * (size_t)tiles_max * kBirthsPerTileMin);
        d.bcnt = (int32_t*)A(4ull * tiles_max);
        int64_t slots = 0;
        for (int s = 0; s < S; ++s) slots += ctx->grid_cap[s];
        d.evr = (uint4*)A(16ull * slots);
        d.evq = (uint4*)A(16ull * slots);
        d.evg = (uint32_t*)A(4ull * kMaxPushGrid);
        d.ccnt = (uint32_t*)A(4ull * tiles_max);
        d.tick = (unsigned long long*)A(8);
        d.ke_part = (double*)A(8ull * tiles_max);
        ctx->poisson_scratch = (double*)A(8ull * 3 * nodes_max);
    }
    if (rc != PIC_OK) {
        pic_free(ctx);
        return rc;
    }
    std::vector<SegState> ss((size_t)B * S);
    std::memset(ss.data(), 0, ss.size() * sizeof(SegState));
    for (int b = 0; b < B; ++b)
        for (int s = 0; s < S; ++s) {
            const pic_species_cfg& sp = cfg[b].species[s];
            const int64_t n = sp.load == PIC_LOAD_NONE ? 0 : sp.n_init;
            ss[b * S + s].count = n;
            ss[b * S + s].live = n;
            ss[b * S + s].next_id = (uint32_t)n;
        }
    std::vector<DisState> ds(B);
    std::memset(ds.data(), 0, ds.size() * sizeof(DisState));
    for (int b = 0; b < B; ++b) ds[b].pw_next = ~0ull;     // no flux sampled yet
    hipStream_t st = ctx->stream;
    bool ok = hipMemcpy(d.segc, ctx->segc.data(), sizeof(SegConst) * B * S, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(d.segs, ss.data(), sizeof(SegState) * B * S, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(d.disc, ctx->disc.data(), sizeof(DisConst) * B, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(d.diss, ds.data(), sizeof(DisState) * B, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemsetAsync(d.acc, 0, 8ull * B * S * kRep * nodes_max, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.cnt, 0, 8ull * B * S * kRep * C_N, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.eacc, 0, 8ull * B * nodes_max, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.macc, 0, 8ull * B * S * 2 * nodes_max, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.pavg, 0, 8ull * B * S * kPow * nodes_max, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.gprev, 0, 8ull * B * S * nodes_max, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.wen, 0, 8ull * B * S * 2, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.avg, 0, 8ull * B * (S + 2) * nodes_max, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.eepf, 0, 8ull * B * 2 * kEepfBins, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.wedf, 0, 8ull * B * S * 2 * kEepfBins, st) == hipSuccess;
    for (int g = 0; g < B * S && ok; ++g)
        for (int k = 0; k < 2 && ok; ++k)
            if (ctx->segc[g].z[k])
                ok = hipMemsetAsync(ctx->segc[g].z[k], 0, 8ull * pad_cap(ctx->segc[g].cap), st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.bcnt, 0, 4ull * tiles_max, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.evg, 0, 4ull * kMaxPushGrid, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.tick, 0, 8, st) == hipSuccess;
    ok = ok && hipMemsetAsync(d.ke_part, 0, 8ull * tiles_max, st) == hipSuccess;
    for (int b = 0; b < B && ok; ++b)
        for (int s = 0; s < S && ok; ++s) {
            const pic_species_cfg& sp = cfg[b].species[s];
            LoadArgs la{};
            la.d = d;
            la.b = b;
            la.s = s;
            la.n = sp.load == PIC_LOAD_NONE ? 0 : sp.n_init;
            la.load = sp.load;
            la.vth = sp.vth;
            for (int k = 0; k < 3; ++k) la.drift[k] = sp.drift[k];
            la.perturb_eps = cfg[b].perturb_eps;
            la.perturb_mode = cfg[b].perturb_mode;
            ok = launch_load(la, st) == hipSuccess;
        }
    if (ok) ok = solve_after_deposit(ctx, -1) == PIC_OK;
    if (ok) ok = launch_halfstep(d, -1, max_count_of(ctx, -1), st) == hipSuccess;
    if (ok) ok = hipStreamSynchronize(st) == hipSuccess;
    if (!ok) {
        pic_free(ctx);
        return PIC_EHIP;
    }
    *out = ctx;
    return PIC_OK;
}

pic_status pic_load_xsec(pic_ctx* ctx, int32_t batch, int32_t species, int32_t kind, double threshold,
                         int32_t n, const double* energy, const double* sigma)
{
    if (!ctx || !energy || !sigma || n < 2) return PIC_EINVAL;
    if (batch < -1 || batch >= ctx->B || species < 0 || species >= ctx->S) return PIC_EINVAL;
    if (kind < PIC_XS_ELASTIC || kind > PIC_XS_ION_ISO || !(threshold >= 0.0)) return PIC_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!(energy[i] > 0.0) || !std::isfinite(energy[i]) || !(sigma[i] >= 0.0) || !std::isfinite(sigma[i]))
            return PIC_EINVAL;
        if (i > 0 && !(energy[i] > energy[i - 1])) return PIC_EINVAL;
    }
    if (kind == PIC_XS_IONIZATION && species != 0) return PIC_EINVAL;
    const int b0 = batch < 0 ? 0 : batch, b1 = batch < 0 ? ctx->B : batch + 1;
    for (int b = b0; b < b1; ++b) {
        const pic_config& c = ctx->cfg[b];
        const SegHost& h = ctx->segh[b * ctx->S + species];
        if (!(c.gas_density > 0.0) || !(c.gas_mass > 0.0)) return PIC_EINVAL;
        if ((int)h.tabs.size() >= kMaxChan) return PIC_EINVAL;
        if (!h.tabs.empty() && electron_kind(h.tabs[0].kind) != electron_kind(kind)) return PIC_EINVAL;
    }
    pic_status rc = hip_st(hipStreamSynchronize(ctx->stream));
    for (int b = b0; b < b1 && rc == PIC_OK; ++b) {
        SegHost& h = ctx->segh[b * ctx->S + species];
        Table t;
        t.kind = kind;
        t.th = threshold;
        t.e.assign(energy, energy + n);
        t.s.assign(sigma, sigma + n);
        h.tabs.push_back(t);
        rc = build_xs(ctx, b, species);
        if (rc == PIC_OK) rc = upload_segc(ctx, b * ctx->S + species);
    }
    return rc;
}

pic_status pic_config_tiles(pic_ctx* ctx, int32_t ppt, int32_t threads, int32_t sort_every,
                            int32_t compact_every)
{
    if (!ctx || (ppt != 1 && ppt != 2 && ppt != 4 && ppt != 8) ||
        (threads != 256 && threads != 512 && threads != 1024) || sort_every < 0 || compact_every < 1 ||
        compact_every > 1024)
        return PIC_EINVAL;
    pic_status rc = hip_st(hipStreamSynchronize(ctx->stream));
    if (rc != PIC_OK) return rc;
    if (sort_every > 0 && !ctx->sort_scratch) {
        int64_t tiles = 0;
        for (int s = 0; s < ctx->S; ++s) {
            int64_t ts = 0;
            for (int b = 0; b < ctx->B; ++b) ts += sort_tiles_for(pad_cap(ctx->segc[b * ctx->S + s].cap));
            tiles = std::max(tiles, ts);
        }
        ctx->sort_tiles = tiles;
        ctx->sort_scratch_bytes = sort_scratch_bytes(tiles, ctx->B, ctx->d.cells_max);
        ctx->sort_scratch = dev_alloc(ctx, ctx->sort_scratch_bytes);
        if (!ctx->sort_scratch) return PIC_ENOMEM;
    }
    ctx->ppt = ppt;
    ctx->threads = threads;
    ctx->sort_every = sort_every;
    ctx->steps_since_sort = 0;
    ctx->compact_every = compact_every;
    ctx->steps_since_compact = 0;
    return rc;
}

pic_status pic_config_events(pic_ctx* ctx, int32_t in_push)
{
    if (!ctx || (in_push != 0 && in_push != 1)) return PIC_EINVAL;
    pic_status rc = hip_st(hipStreamSynchronize(ctx->stream));
    if (rc != PIC_OK) return rc;
    ctx->events_in_push = in_push;
    return rc;
}

pic_status pic_set_diag(pic_ctx* ctx, int32_t enable, double eepf_emax_eV)
{
    if (!ctx || !(eepf_emax_eV > 0.0) || !std::isfinite(eepf_emax_eV)) return PIC_EINVAL;
    ctx->diag = enable ? 1 : 0;
    ctx->eepf_emax = eepf_emax_eV;
    return PIC_OK;
}

pic_status pic_set_wall_edf(pic_ctx* ctx, int32_t species, double emax_eV)
{
    if (!ctx || species < 0 || species >= ctx->S || !(emax_eV > 0.0) || !std::isfinite(emax_eV))
        return PIC_EINVAL;
    pic_status rc = hip_st(hipStreamSynchronize(ctx->stream));
    for (int b = 0; b < ctx->B && rc == PIC_OK; ++b) {
        ctx->segc[b * ctx->S + species].wedf_inv_bin = (float)(kEepfBins / emax_eV);
        rc = upload_segc(ctx, b * ctx->S + species);
    }
    if (rc == PIC_OK) ctx->wedf_emax[species] = emax_eV;
    return rc;
}

namespace {

struct StepPlan {
    PushArgs pa{};
    int ppt = 4, threads = 256;
    bool general = false;
    bool fuse = false;                   // the push does the events (no events launch)
    int64_t grid = 1;
    EvArgs ea{};
    int64_t ev_grid = 1;
    FinArgs fa{};
    uint64_t key = 0;
};

pic_status plan_step(pic_ctx* ctx, StepPlan& p)
{
    const int S = ctx->S, B = ctx->B;
    int nn_max = 0, nc_max = 0;
    for (int b = 0; b < B; ++b) {
        nn_max = std::max(nn_max, ctx->disc[b].n_nodes);
        nc_max = std::max(nc_max, ctx->disc[b].n_cells);
    }
    // one launch for every segment: the general kernel as soon as any segment
    // can lose, gain or collide particles; tile shape; persistent grid
    const size_t lds = push_lds_bytes(nn_max, nc_max, ctx->diag);
    if (lds > 65536) return PIC_EINVAL;
    p.ppt = ctx->ppt;
    p.threads = ctx->threads;
    p.general = false;
    for (int g = 0; g < B * S; ++g) {
        const SegConst& sc = ctx->segc[g];
        if (sc.compacts || sc.nch > 0 || sc.emits || sc.renew_lz > 0.0) p.general = true;
    }
    push_shape(p.ppt, p.threads, p.general);
    p.fuse = ctx->events_in_push && push_fusable(p.ppt, p.threads, p.general);
    const int T = p.threads * p.ppt;
    int64_t tiles = 0;
    for (int g = 0; g < B * S; ++g) tiles += (pad_cap(ctx->segc[g].cap) + T - 1) / T;
    const int64_t resident = (int64_t)push_occupancy(p.ppt, p.threads, p.general, p.fuse, lds) * ctx->n_cu;
    p.grid = std::max<int64_t>(1, std::min(std::min(tiles, resident), (int64_t)kMaxPushGrid));
    PushArgs& pa = p.pa;
    pa.d = ctx->d;
    pa.diag = ctx->diag;
    pa.eepf_inv_bin = (float)(kEepfBins / ctx->eepf_emax);
    pa.nodes_max_dyn = nn_max;
    pa.cells_max_dyn = nc_max;
    uint64_t key = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
    mix((uint64_t)ctx->diag);
    {
        uint32_t bits;
        std::memcpy(&bits, &pa.eepf_inv_bin, 4);
        mix((uint64_t)bits);    // a captured step holds the bin width
    }
    mix((uint64_t)p.ppt);
    mix((uint64_t)p.threads);
    mix((uint64_t)p.general);
    mix((uint64_t)p.fuse);
    mix((uint64_t)p.grid);
    p.fa.d = ctx->d;
    p.fa.mode = kFinStep;
    p.fa.diag = ctx->diag;
    p.fa.only_b = -1;
    p.fa.births_per_tile = p.general ? T / kBirthsDiv : 0;
    p.ea.d = ctx->d;
    p.ea.T = T;
    p.ea.push_grid = (int32_t)p.grid;
    p.ea.births_per_tile = T / kBirthsDiv;
    p.ea.diag = ctx->diag;
    p.ea.eepf_inv_bin = pa.eepf_inv_bin;
    p.ev_grid = std::max<int64_t>(1, std::min(tiles, (int64_t)events_occupancy() * ctx->n_cu));
    mix((uint64_t)p.ev_grid);
    p.fa.eepf_inv_bin = pa.eepf_inv_bin;
    mix((uint64_t)ctx->sort_every);
    mix((uint64_t)ctx->compact_every);
    p.key = key;
    return PIC_OK;
}

// queue `n` steps on stream st; `prof` wraps every launch in an event pair
pic_status enqueue_steps(pic_ctx* ctx, const StepPlan& p, int n, hipStream_t st, bool prof)
{
    for (int it = 0; it < n; ++it) {
        if (ctx->sort_every > 0 && ++ctx->steps_since_sort >= ctx->sort_every) {
            ctx->steps_since_sort = 0;
            for (int s = 0; s < ctx->S; ++s)
                if (launch_sort(ctx->d, s, ctx->sort_tiles, ctx->sort_scratch, ctx->sort_scratch_bytes, st) !=
                    hipSuccess)
                    return PIC_EHIP;
        }
        const int pp = prof ? prof_begin(ctx) : -1;
        if (launch_push(p.pa, p.ppt, p.threads, p.general, p.fuse, p.grid, st) != hipSuccess) return PIC_EHIP;
        prof_end(ctx, pp, 0);
        if (p.general && !p.fuse) {
            const int pv = prof ? prof_begin(ctx) : -1;
            if (launch_events(p.ea, p.ev_grid, st) != hipSuccess) return PIC_EHIP;
            prof_end(ctx, pv, 1);
        }
        const int pe = prof ? prof_begin(ctx) : -1;
        if (launch_finalize(p.fa, st) != hipSuccess) return PIC_EHIP;
        prof_end(ctx, pe, -1);
        // the general kernel leaves holes where particles were absorbed
        if (p.general && ++ctx->steps_since_compact >= ctx->compact_every) {
            ctx->steps_since_compact = 0;
            if (launch_compact(ctx->d, ctx->compact_tiles, ctx->n_cu, st) != hipSuccess) return PIC_EHIP;
        }
        if (prof && ctx->ev_used + 8 > 4096) prof_collect(ctx);
    }
    return PIC_OK;
}

void drop_graph(pic_ctx* ctx)
{
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    ctx->gexec = nullptr;
    ctx->g_steps = 0;
}

// capture `n` steps into a replayable graph (on a private capture stream)
pic_status capture_steps(pic_ctx* ctx, const StepPlan& p, int n)
{
    drop_graph(ctx);
    if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return PIC_EHIP;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return PIC_EHIP;
    const int64_t saved = ctx->steps_since_sort, saved_c = ctx->steps_since_compact;
    const pic_status rc = enqueue_steps(ctx, p, n, ctx->cap_stream, false);
    ctx->steps_since_sort = saved;
    ctx->steps_since_compact = saved_c;
    const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (rc != PIC_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc != PIC_OK ? rc : PIC_EHIP;
    }
    const hipError_t ei = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        ctx->gexec = nullptr;
        return PIC_EHIP;
    }
    ctx->g_steps = n;
    ctx->g_key = p.key;
    return PIC_OK;
}

constexpr int kGraphSteps = 32;
constexpr int kGraphMaxSteps = 1024;

int64_t gcd64(int64_t a, int64_t b)
{
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// steps of the captured chunk: a multiple of 32 that every periodic
// interval (sort, compaction) divides, so each replay sorts and compacts at
// the same steps; 0 when that would exceed kGraphMaxSteps
int graph_chunk(const pic_ctx* ctx, const StepPlan& p)
{
    int64_t L = kGraphSteps;
    if (ctx->sort_every > 0) L = L / gcd64(L, ctx->sort_every) * ctx->sort_every;
    if (p.general) L = L / gcd64(L, ctx->compact_every) * ctx->compact_every;
    return L <= kGraphMaxSteps ? (int)L : 0;
}

}  // namespace

pic_status pic_step(pic_ctx* ctx, int32_t n_steps)
{
    if (!ctx || n_steps < 0) return PIC_EINVAL;
    StepPlan p;
    pic_status rc = plan_step(ctx, p);
    if (rc != PIC_OK) return rc;
    hipStream_t st = ctx->stream;
    int left = n_steps;
    // direct steps until the sort and compaction counters are back at zero,
    // so that every replay of the captured chunk sorts and compacts at the
    // same steps
    auto aligned = [&]() {
        return (ctx->sort_every == 0 || ctx->steps_since_sort == 0) &&
               (!p.general || ctx->steps_since_compact == 0);
    };
    const int chunk = graph_chunk(ctx, p);
    while (chunk > 0 && ctx->use_graph && !ctx->prof && !aligned() && left > 0) {
        rc = enqueue_steps(ctx, p, 1, st, false);
        if (rc != PIC_OK) return rc;
        --left;
    }
    // replays of a captured chunk; the intervals divide the chunk
    const bool graph_ok = ctx->use_graph && !ctx->prof && chunk > 0 && aligned();
    if (graph_ok && left >= chunk) {
        if (!ctx->gexec || ctx->g_key != p.key || ctx->g_steps != chunk) {
            rc = capture_steps(ctx, p, chunk);
            if (rc != PIC_OK) return rc;
        }
        while (left >= chunk) {
            if (hipGraphLaunch(ctx->gexec, st) != hipSuccess) return PIC_EHIP;
            left -= chunk;
            ctx->graph_replays += 1;
            ctx->graph_steps += chunk;
        }
    }
    return enqueue_steps(ctx, p, left, st, ctx->prof != 0);
}

pic_status pic_retire(pic_ctx* ctx, int32_t batch, int32_t retired)
{
    if (!ctx || batch < 0 || batch >= ctx->B) return PIC_EINVAL;
    const int32_t v = retired ? 1 : 0;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return PIC_EHIP;
    return hip_st(hipMemcpy(&ctx->d.diss[batch].retired, &v, sizeof(v), hipMemcpyHostToDevice));
}

pic_status pic_thin(pic_ctx* ctx, int32_t species, int64_t above, int64_t keep)
{
    if (!ctx || species < 0 || species >= ctx->S || keep < 0 || keep > above) return PIC_EINVAL;
    int64_t max_count = 0;
    for (int b = 0; b < ctx->B; ++b) max_count = std::max(max_count, pad_cap(ctx->segc[b * ctx->S + species].cap));
    return launch_thin(ctx->d, species, above, keep, max_count, ctx->compact_tiles, ctx->n_cu, ctx->stream) ==
                   hipSuccess
               ? PIC_OK
               : PIC_EHIP;
}

pic_status pic_sort(pic_ctx* ctx)
{
    if (!ctx) return PIC_EINVAL;
    if (!ctx->sort_scratch) {
        int64_t tiles = 0;
        for (int s = 0; s < ctx->S; ++s) {
            int64_t ts = 0;
            for (int b = 0; b < ctx->B; ++b) ts += sort_tiles_for(pad_cap(ctx->segc[b * ctx->S + s].cap));
            tiles = std::max(tiles, ts);
        }
        ctx->sort_tiles = tiles;
        ctx->sort_scratch_bytes = sort_scratch_bytes(tiles, ctx->B, ctx->d.cells_max);
        ctx->sort_scratch = dev_alloc(ctx, ctx->sort_scratch_bytes);
        if (!ctx->sort_scratch) return PIC_ENOMEM;
    }
    for (int s = 0; s < ctx->S; ++s)
        if (launch_sort(ctx->d, s, ctx->sort_tiles, ctx->sort_scratch, ctx->sort_scratch_bytes, ctx->stream) !=
            hipSuccess)
            return PIC_EHIP;
    return PIC_OK;
}

pic_status pic_sort_noalloc(pic_ctx* ctx)
{
    if (!ctx) return PIC_EINVAL;
    void* ptr = noalloc_scratch(ctx->device);
    if (!ptr) return PIC_ESTATE;
    int64_t tiles = 0;
    for (int s = 0; s < ctx->S; ++s) {
        int64_t ts = 0;
        for (int b = 0; b < ctx->B; ++b) ts += sort_tiles_for(pad_cap(ctx->segc[b * ctx->S + s].cap));
        tiles = std::max(tiles, ts);
    }
    if (sort_scratch_bytes(tiles, ctx->B, ctx->d.cells_max) > (size_t)PIC_NOALLOC_SCRATCH_BYTES) return PIC_ESCRATCH;
    for (int s = 0; s < ctx->S; ++s)
        if (launch_sort(ctx->d, s, tiles, ptr, PIC_NOALLOC_SCRATCH_BYTES, ctx->stream) != hipSuccess) return PIC_EHIP;
    return PIC_OK;
}

pic_status pic_use_graphs(pic_ctx* ctx, int32_t enable)
{
    if (!ctx) return PIC_EINVAL;
    ctx->use_graph = enable ? 1 : 0;
    if (!enable) drop_graph(ctx);
    return PIC_OK;
}

pic_status pic_profile(pic_ctx* ctx, int32_t enable)
{
    if (!ctx) return PIC_EINVAL;
    prof_collect(ctx);
    ctx->prof = enable ? 1 : 0;
    if (enable) {
        ctx->push_ms = ctx->push_n = 0.0;
        ctx->fin_ms = ctx->fin_n = 0.0;
        ctx->ev_ms = ctx->ev_n = 0.0;
    }
    return PIC_OK;
}

pic_status pic_sync(pic_ctx* ctx)
{
    if (!ctx) return PIC_EINVAL;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return PIC_EHIP;
    std::vector<DisState> ds(ctx->B);
    if (hipMemcpy(ds.data(), ctx->d.diss, sizeof(DisState) * ctx->B, hipMemcpyDeviceToHost) != hipSuccess)
        return PIC_EHIP;
    uint32_t f = 0;
    for (const auto& x : ds) f |= x.flags;
    return flags_status(f);
}

pic_status pic_poisson(pic_ctx* ctx, int32_t batch, double t_s, const double* rho_in, double* phi_out,
                       double* e_out)
{
    if (!ctx || batch < 0 || batch >= ctx->B) return PIC_EINVAL;
    const int nn = ctx->disc[batch].n_nodes;
    const size_t nm = ctx->d.nodes_max;
    double* rho_d = ctx->poisson_scratch;
    double* phi_d = rho_d + nm;
    double* e_d = phi_d + nm;
    hipStream_t st = ctx->stream;
    if (hipStreamSynchronize(st) != hipSuccess) return PIC_EHIP;
    hipError_t e;
    if (rho_in) e = hipMemcpy(rho_d, rho_in, nn * sizeof(double), hipMemcpyHostToDevice);
    else e = hipMemcpy(rho_d, ctx->d.rho + (size_t)batch * nm, nn * sizeof(double), hipMemcpyDeviceToDevice);
    if (e != hipSuccess) return PIC_EHIP;
    FinArgs fa{};
    fa.d = ctx->d;
    fa.mode = kFinExternal;
    fa.only_b = batch;
    fa.t_ext = t_s;
    fa.rho_ext = rho_d;
    fa.phi_out = phi_d;
    fa.e_out = e_d;
    if (launch_finalize(fa, st) != hipSuccess) return PIC_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return PIC_EHIP;
    if (phi_out && hipMemcpy(phi_out, phi_d, nn * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return PIC_EHIP;
    if (e_out && hipMemcpy(e_out, e_d, nn * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return PIC_EHIP;
    return PIC_OK;
}

pic_status pic_set_windows(pic_ctx* ctx, int32_t batch, int64_t steps)
{
    if (!ctx || batch < 0 || batch >= ctx->B || steps < 0) return PIC_EINVAL;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return PIC_EHIP;
    DisState ds;
    if (hipMemcpy(&ds, ctx->d.diss + batch, sizeof(DisState), hipMemcpyDeviceToHost) != hipSuccess) return PIC_EHIP;
    ds.win_len = steps;
    ds.win_start = (int64_t)ds.step;
    ds.nwin = 0;
    ds.avg_samples = 0.0;
    const size_t nm = ctx->d.nodes_max;
    if (hipMemset(ctx->d.avg + (size_t)batch * (ctx->S + 2) * nm, 0, 8ull * (ctx->S + 2) * nm) != hipSuccess)
        return PIC_EHIP;
    return hip_st(hipMemcpy(ctx->d.diss + batch, &ds, sizeof(DisState), hipMemcpyHostToDevice));
}

pic_status pic_get_windows(pic_ctx* ctx, int32_t batch, int64_t first, int32_t count, double* out,
                           int64_t* n_done)
{
    if (!ctx || batch < 0 || batch >= ctx->B || first < 0 || count < 0 || (count > 0 && !out)) return PIC_EINVAL;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return PIC_EHIP;
    DisState ds;
    if (hipMemcpy(&ds, ctx->d.diss + batch, sizeof(DisState), hipMemcpyDeviceToHost) != hipSuccess) return PIC_EHIP;
    if (n_done) *n_done = ds.nwin;
    if (count == 0) return PIC_OK;
    if (first + count > ds.nwin || first < ds.nwin - kWindowRing) return PIC_EINVAL;
    const int S = ctx->S;
    const int nn = ctx->disc[batch].n_nodes;
    const size_t nm = ctx->d.nodes_max, stride = 1 + (size_t)(S + 2) * nm;
    std::vector<double> w(stride);
    for (int32_t k = 0; k < count; ++k) {
        const int64_t idx = first + k;
        if (hipMemcpy(w.data(), ctx->d.wring + ((size_t)batch * kWindowRing + (size_t)(idx % kWindowRing)) * stride,
                      stride * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return PIC_EHIP;
        double* o = out + (size_t)k * (1 + (size_t)(S + 2) * nn);
        const double ns = w[0];
        o[0] = ns;
        for (int r = 0; r < S + 2; ++r)
            for (int i = 0; i < nn; ++i) {
                double v = w[1 + (size_t)r * nm + i];
                if (r == S + 1) {
                    const double ne = w[1 + i];
                    v = ne > 0.0 ? v / ne : 0.0;          // <eps> = sum(n eps) / sum(n)
                } else if (ns > 0.0) {
                    v /= ns;
                }
                o[1 + (size_t)r * nn + i] = v;
            }
    }
    return PIC_OK;
}

pic_status pic_set_circuit(pic_ctx* ctx, int32_t batch, double q)
{
    if (!ctx || batch < 0 || batch >= ctx->B || !std::isfinite(q)) return PIC_EINVAL;
    const DisConst& dc = ctx->disc[batch];
    if (dc.bc == PIC_BC_PERIODIC || !dc.field_solve || dc.drive == PIC_DRIVE_VOLTAGE) return PIC_EINVAL;
    hipStream_t st = ctx->stream;
    if (hipStreamSynchronize(st) != hipSuccess) return PIC_EHIP;
    const int S = ctx->S;
    std::vector<unsigned long long> cr((size_t)S * kRep * C_N);
    DisState ds;
    if (hipMemcpy(cr.data(), ctx->d.cnt + (size_t)batch * S * kRep * C_N, cr.size() * 8, hipMemcpyDeviceToHost) !=
            hipSuccess ||
        hipMemcpy(&ds, ctx->d.diss + batch, sizeof(DisState), hipMemcpyDeviceToHost) != hipSuccess)
        return PIC_EHIP;
    ds.qbase = q - source_charge(dc, (double)ds.step * dc.dt) - collected_charge(dc, cr.data(), S);
    ds.circ_init = 1;
    if (hipMemcpy(ctx->d.diss + batch, &ds, sizeof(DisState), hipMemcpyHostToDevice) != hipSuccess) return PIC_EHIP;
    if (hipMemset(ctx->d.acc + (size_t)batch * S * kRep * ctx->d.nodes_max, 0, 8ull * S * kRep * ctx->d.nodes_max) !=
        hipSuccess)
        return PIC_EHIP;
    pic_status rc = solve_after_deposit(ctx, batch);
    if (rc != PIC_OK) return rc;
    return hip_st(hipStreamSynchronize(st));
}

pic_status pic_get_axial(pic_ctx* ctx, int32_t batch, int32_t species, int64_t cap, double* z, int64_t* n_out)
{
    if (!ctx || batch < 0 || batch >= ctx->B || species < 0 || species >= ctx->S) return PIC_EINVAL;
    const int idx = batch * ctx->S + species;
    const SegConst& sc = ctx->segc[idx];
    if (!sc.z[0]) return PIC_EINVAL;
    int64_t n = 0;
    uint32_t nid = 0;
    // the particles' own read compacts the store first, so z is in canonical order
    pic_status rc = pic_get_particles(ctx, batch, species, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                                      nullptr, &n, &nid);
    if (rc != PIC_OK) return rc;
    if (n_out) *n_out = n;
    if (!z || cap < n) return PIC_OK;
    SegState ss;
    if (hipMemcpy(&ss, ctx->d.segs + idx, sizeof(SegState), hipMemcpyDeviceToHost) != hipSuccess) return PIC_EHIP;
    if (ss.count != ss.live) {
        if (launch_compact(ctx->d, ctx->compact_tiles, ctx->n_cu, ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess ||
            hipMemcpy(&ss, ctx->d.segs + idx, sizeof(SegState), hipMemcpyDeviceToHost) != hipSuccess)
            return PIC_EHIP;
        if (ss.count != ss.live) return PIC_ESTATE;
    }
    return hip_st(hipMemcpy(z, sc.z[ss.parity], (size_t)ss.count * 8, hipMemcpyDeviceToHost));
}

pic_status pic_set_axial(pic_ctx* ctx, int32_t batch, int32_t species, int64_t n, const double* z)
{
    if (!ctx || batch < 0 || batch >= ctx->B || species < 0 || species >= ctx->S || n < 0) return PIC_EINVAL;
    const int idx = batch * ctx->S + species;
    const SegConst& sc = ctx->segc[idx];
    if (!sc.z[0] || (n > 0 && !z)) return PIC_EINVAL;
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(z[k])) return PIC_EINVAL;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return PIC_EHIP;
    SegState ss;
    if (hipMemcpy(&ss, ctx->d.segs + idx, sizeof(SegState), hipMemcpyDeviceToHost) != hipSuccess) return PIC_EHIP;
    if (ss.count != ss.live) {
        if (launch_compact(ctx->d, ctx->compact_tiles, ctx->n_cu, ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess ||
            hipMemcpy(&ss, ctx->d.segs + idx, sizeof(SegState), hipMemcpyDeviceToHost) != hipSuccess)
            return PIC_EHIP;
        if (ss.count != ss.live) return PIC_ESTATE;
    }
    if (n != ss.live) return PIC_EINVAL;
    if (n == 0) return PIC_OK;
    return hip_st(hipMemcpy(sc.z[ss.parity], z, (size_t)n * 8, hipMemcpyHostToDevice));
}

pic_status pic_get_particles(pic_ctx* ctx, int32_t batch, int32_t species, int64_t cap, int32_t* cell,
                             float* off, float* vx, float* vy, float* vz, uint32_t* id, int64_t* n_out,
                             uint32_t* next_id)
{
    if (!ctx || batch < 0 || batch >= ctx->B || species < 0 || species >= ctx->S) return PIC_EINVAL;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return PIC_EHIP;
    const int idx = batch * ctx->S + species;
    SegState ss;
    if (hipMemcpy(&ss, ctx->d.segs + idx, sizeof(SegState), hipMemcpyDeviceToHost) != hipSuccess) return PIC_EHIP;
    if (n_out) *n_out = ss.live;
    if (next_id) *next_id = ss.next_id;
    if (!cell && !off && !vx && !vy && !vz && !id) return PIC_OK;
    if (cap < ss.live) return PIC_EINVAL;
    if (ss.count != ss.live) {
        // holes first: the copy holds the live particles in their order
        if (launch_compact(ctx->d, ctx->compact_tiles, ctx->n_cu, ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess ||
            hipMemcpy(&ss, ctx->d.segs + idx, sizeof(SegState), hipMemcpyDeviceToHost) != hipSuccess)
            return PIC_EHIP;
        if (ss.count != ss.live) return PIC_ESTATE;
    }
    const SegConst& sc = ctx->segc[idx];
    const int p = ss.parity;
    const size_t nb = (size_t)ss.count * 4;
    bool ok = true;
    if (cell) ok = ok && hipMemcpy(cell, sc.cell[p], nb, hipMemcpyDeviceToHost) == hipSuccess;
    if (off) ok = ok && hipMemcpy(off, sc.off[p], nb, hipMemcpyDeviceToHost) == hipSuccess;
    if (vx) ok = ok && hipMemcpy(vx, sc.vx[p], nb, hipMemcpyDeviceToHost) == hipSuccess;
    if (vy) ok = ok && hipMemcpy(vy, sc.vy[p], nb, hipMemcpyDeviceToHost) == hipSuccess;
    if (vz) ok = ok && hipMemcpy(vz, sc.vz[p], nb, hipMemcpyDeviceToHost) == hipSuccess;
    if (id) ok = ok && hipMemcpy(id, sc.id[p], nb, hipMemcpyDeviceToHost) == hipSuccess;
    return ok ? PIC_OK : PIC_EHIP;
}

pic_status pic_set_particles(pic_ctx* ctx, int32_t batch, int32_t species, int64_t n, const int32_t* cell,
                             const float* off, const float* vx, const float* vy, const float* vz,
                             const uint32_t* id, uint32_t next_id, uint64_t step)
{
    if (!ctx || batch < 0 || batch >= ctx->B || species < 0 || species >= ctx->S || n < 0) return PIC_EINVAL;
    const int idx = batch * ctx->S + species;
    const SegConst& sc = ctx->segc[idx];
    if (n > sc.cap || (n > 0 && (!cell || !off || !vx || !vy || !vz || !id))) return PIC_EINVAL;
    const int nc = ctx->disc[batch].n_cells;
    for (int64_t k = 0; k < n; ++k) {
        if (cell[k] < 0 || cell[k] >= nc || !(off[k] >= 0.0f && off[k] < 1.0f)) return PIC_EINVAL;
        if (!std::isfinite(vx[k]) || !std::isfinite(vy[k]) || !std::isfinite(vz[k])) return PIC_ENUMERIC;
    }
    hipStream_t st = ctx->stream;
    if (hipStreamSynchronize(st) != hipSuccess) return PIC_EHIP;
    SegState ss;
    if (hipMemcpy(&ss, ctx->d.segs + idx, sizeof(SegState), hipMemcpyDeviceToHost) != hipSuccess) return PIC_EHIP;
    const int p = ss.parity;
    const size_t nb = (size_t)n * 4;
    bool ok = true;
    if (n > 0) {
        ok = ok && hipMemcpy(sc.cell[p], cell, nb, hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(sc.off[p], off, nb, hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(sc.vx[p], vx, nb, hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(sc.vy[p], vy, nb, hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(sc.vz[p], vz, nb, hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(sc.id[p], id, nb, hipMemcpyHostToDevice) == hipSuccess;
        if (sc.z[p]) ok = ok && hipMemset(sc.z[p], 0, 2 * nb) == hipSuccess;
    }
    ss.count = n;
    ss.live = n;
    ss.dead = 0;
    ss.staged = 0;
    ss.next_id = next_id;
    ss.ntiles = 0;
    ok = ok && hipMemcpy(ctx->d.segs + idx, &ss, sizeof(SegState), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) return PIC_EHIP;
    // the whole context moves to `step`
    std::vector<DisState> ds(ctx->B);
    if (hipMemcpy(ds.data(), ctx->d.diss, sizeof(DisState) * ctx->B, hipMemcpyDeviceToHost) != hipSuccess)
        return PIC_EHIP;
    for (auto& x : ds) x.step = step;
    ds[batch].circ_init = 0;            // new particles: the circuit restarts at the next solve
    if (hipMemcpy(ctx->d.diss, ds.data(), sizeof(DisState) * ctx->B, hipMemcpyHostToDevice) != hipSuccess)
        return PIC_EHIP;
    if (hipMemset(ctx->d.acc + (size_t)batch * ctx->S * kRep * ctx->d.nodes_max, 0,
                  8ull * ctx->S * kRep * ctx->d.nodes_max) != hipSuccess)
        return PIC_EHIP;
    pic_status rc = solve_after_deposit(ctx, batch);
    if (rc != PIC_OK) return rc;
    return hip_st(hipStreamSynchronize(st));
}

pic_status pic_load_profiles(pic_ctx* ctx, int32_t batch, int32_t m, const double* density, const double* temp_eV,
                             const int64_t* n)
{
    if (!ctx || batch < 0 || batch >= ctx->B || m < 2 || m > kMaxCells + 1 || !density || !temp_eV || !n)
        return PIC_EINVAL;
    const int S = ctx->S;
    const pic_config& c = ctx->cfg[batch];
    const double h = c.length / (double)(m - 1);
    // per species: density, its running integral, temperature
    std::vector<double> tab((size_t)3 * m * S);
    for (int s = 0; s < S; ++s) {
        const double* ds = density + (size_t)s * m;
        const double* ts = temp_eV + (size_t)s * m;
        double* dd = tab.data() + (size_t)3 * m * s;
        double* cum = dd + m;
        double* tt = cum + m;
        if (n[s] < 0 || n[s] > ctx->segc[batch * S + s].cap) return PIC_EINVAL;
        for (int i = 0; i < m; ++i) {
            if (!(ds[i] >= 0.0) || !std::isfinite(ds[i]) || !(ts[i] >= 0.0) || !std::isfinite(ts[i]))
                return PIC_EINVAL;
            dd[i] = ds[i];
            tt[i] = ts[i];
            cum[i] = i == 0 ? 0.0 : cum[i - 1] + 0.5 * (ds[i - 1] + ds[i]) * h;
        }
        if (n[s] > 0 && !(cum[m - 1] > 0.0)) return PIC_EINVAL;
    }
    hipStream_t st = ctx->stream;
    if (hipStreamSynchronize(st) != hipSuccess) return PIC_EHIP;
    double* dev = (double*)dev_alloc(ctx, sizeof(double) * tab.size());
    if (!dev) return PIC_ENOMEM;
    bool ok = hipMemcpy(dev, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice) == hipSuccess;
    std::vector<SegState> ss(S);
    ok = ok && hipMemcpy(ss.data(), ctx->d.segs + (size_t)batch * S, sizeof(SegState) * S, hipMemcpyDeviceToHost) ==
                   hipSuccess;
    for (int s = 0; s < S && ok; ++s) {
        ProfileArgs pa{};
        pa.d = ctx->d;
        pa.b = batch;
        pa.s = s;
        pa.m = m;
        pa.n = n[s];
        pa.dens = dev + (size_t)3 * m * s;
        pa.cum = pa.dens + m;
        pa.temp = pa.cum + m;
        pa.e_over_m = c.e_unit / c.species[s].mass;
        ok = launch_profile_load(pa, st) == hipSuccess;
        const SegConst& zc = ctx->segc[batch * S + s];
        if (ok && zc.z[ss[s].parity] && n[s] > 0)
            ok = hipMemsetAsync(zc.z[ss[s].parity], 0, 8ull * n[s], st) == hipSuccess;
        ss[s].count = ss[s].live = n[s];
        ss[s].dead = 0;
        ss[s].staged = 0;
        ss[s].next_id = (uint32_t)n[s];
        ss[s].ntiles = 0;
    }
    ok = ok && hipMemcpy(ctx->d.segs + (size_t)batch * S, ss.data(), sizeof(SegState) * S, hipMemcpyHostToDevice) ==
                   hipSuccess;
    {
        DisState dsb;
        ok = ok && hipMemcpy(&dsb, ctx->d.diss + batch, sizeof(DisState), hipMemcpyDeviceToHost) == hipSuccess;
        dsb.circ_init = 0;              // new particles: the circuit restarts at the next solve
        ok = ok && hipMemcpy(ctx->d.diss + batch, &dsb, sizeof(DisState), hipMemcpyHostToDevice) == hipSuccess;
    }
    ok = ok && hipMemset(ctx->d.acc + (size_t)batch * S * kRep * ctx->d.nodes_max, 0,
                         8ull * S * kRep * ctx->d.nodes_max) == hipSuccess;
    ok = ok && solve_after_deposit(ctx, batch) == PIC_OK;
    ok = ok && launch_halfstep(ctx->d, batch, max_count_of(ctx, batch), st) == hipSuccess;
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    dev_release(ctx, dev);
    return ok ? PIC_OK : PIC_EHIP;
}

pic_status pic_diag(pic_ctx* ctx, int32_t batch, int32_t what, void* out, size_t out_bytes)
{
    if (!ctx || batch < 0 || batch >= ctx->B) return PIC_EINVAL;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return PIC_EHIP;
    const int S = ctx->S;
    const int nn = ctx->disc[batch].n_nodes;
    const size_t nm = ctx->d.nodes_max;
    std::vector<SegState> ss(S);
    DisState ds;
    std::vector<unsigned long long> cr((size_t)S * kRep * C_N);
    std::vector<unsigned long long> ev((size_t)S * C_N, 0ull);   // counters summed over copies
    if (hipMemcpy(cr.data(), ctx->d.cnt + (size_t)batch * S * kRep * C_N, cr.size() * 8, hipMemcpyDeviceToHost) !=
        hipSuccess)
        return PIC_EHIP;
    for (int s = 0; s < S; ++s)
        for (int r = 0; r < kRep; ++r)
            for (int k = 0; k < C_N; ++k) ev[(size_t)s * C_N + k] += cr[((size_t)s * kRep + r) * C_N + k];
    if (hipMemcpy(ss.data(), ctx->d.segs + (size_t)batch * S, sizeof(SegState) * S, hipMemcpyDeviceToHost) !=
            hipSuccess ||
        hipMemcpy(&ds, ctx->d.diss + batch, sizeof(DisState), hipMemcpyDeviceToHost) != hipSuccess)
        return PIC_EHIP;
    auto need = [&](size_t bytes) { return out && out_bytes >= bytes; };
    auto d2h = [&](void* dst, const void* src, size_t bytes) {
        return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) == hipSuccess;
    };
    bool ok = true;
    switch (what) {
        case PIC_DIAG_COUNTS: {
            if (!need(8 * (4 + 2 * S))) return PIC_EINVAL;
            int64_t* o = (int64_t*)out;
            o[0] = (int64_t)ds.step;
            o[1] = nn;
            o[2] = S;
            o[3] = ds.flags;
            for (int s = 0; s < S; ++s) {
                o[4 + 2 * s] = ss[s].live;
                o[5 + 2 * s] = ss[s].next_id;
            }
            break;
        }
        case PIC_DIAG_RHO:
        case PIC_DIAG_PHI:
        case PIC_DIAG_EFIELD: {
            if (!need(8ull * nn)) return PIC_EINVAL;
            const double* src = what == PIC_DIAG_RHO ? ctx->d.rho : (what == PIC_DIAG_PHI ? ctx->d.phi : ctx->d.ef);
            ok = d2h(out, src + (size_t)batch * nm, 8ull * nn);
            break;
        }
        case PIC_DIAG_DENSITY: {
            if (!need(8ull * S * nn)) return PIC_EINVAL;
            for (int s = 0; s < S && ok; ++s)
                ok = d2h((double*)out + (size_t)s * nn, ctx->d.dens + ((size_t)batch * S + s) * nm, 8ull * nn);
            break;
        }
        case PIC_DIAG_ENERGY: {
            if (!need(8ull * (S + 1))) return PIC_EINVAL;
            double* o = (double*)out;
            for (int s = 0; s < S; ++s) o[s] = ss[s].ke;
            o[S] = ds.fe;
            break;
        }
        case PIC_DIAG_WALL: {
            if (!need(8ull * (2 * S + 2))) return PIC_EINVAL;
            int64_t* o = (int64_t*)out;
            int64_t see0 = 0, see1 = 0;
            for (int s = 0; s < S; ++s) {
                o[2 * s] = (int64_t)ev[(size_t)s * C_N + C_ABS0];
                o[2 * s + 1] = (int64_t)ev[(size_t)s * C_N + C_ABS1];
                see0 += (int64_t)ev[(size_t)s * C_N + C_SEE0];
                see1 += (int64_t)ev[(size_t)s * C_N + C_SEE1];
            }
            o[2 * S] = see0;
            o[2 * S + 1] = see1;
            break;
        }
        case PIC_DIAG_COLL: {
            if (!need(8ull * S * (3 + kMaxChan))) return PIC_EINVAL;
            int64_t* o = (int64_t*)out;
            for (int s = 0; s < S; ++s) {
                int64_t* r = o + (size_t)s * (3 + kMaxChan);
                r[0] = (int64_t)ev[(size_t)s * C_N + C_CAND];
                r[1] = (int64_t)ev[(size_t)s * C_N + C_NULL];
                r[2] = (int64_t)ev[(size_t)s * C_N + C_VIOL];
                for (int k = 0; k < kMaxChan; ++k) r[3 + k] = (int64_t)ev[(size_t)s * C_N + C_COLL + k];
            }
            break;
        }
        case PIC_DIAG_NUMAX: {
            if (!need(8ull * 2 * S)) return PIC_EINVAL;
            double* o = (double*)out;
            for (int s = 0; s < S; ++s) {
                o[s] = ctx->segh[(size_t)batch * S + s].numax;
                o[S + s] = (double)ctx->segh[(size_t)batch * S + s].t32;
            }
            break;
        }
        case PIC_DIAG_FLAGS: {
            if (!need(8)) return PIC_EINVAL;
            *(int64_t*)out = ds.flags;
            const uint32_t z = 0;
            ok = hipMemcpy(&ctx->d.diss[batch].flags, &z, 4, hipMemcpyHostToDevice) == hipSuccess;
            if (!ok) return PIC_EHIP;
            return PIC_OK;
        }
        case PIC_DIAG_AVG: {
            if (!need(8ull * (1 + (size_t)(S + 2) * nn))) return PIC_EINVAL;
            double* o = (double*)out;
            std::vector<double> av((size_t)(S + 2) * nm);
            ok = d2h(av.data(), ctx->d.avg + (size_t)batch * (S + 2) * nm, av.size() * 8);
            const double ns = ds.avg_samples;
            o[0] = ns;
            for (int k = 0; k < S + 2; ++k)
                for (int i = 0; i < nn; ++i) {
                    double v = av[(size_t)k * nm + i];
                    if (k == S + 1) {
                        const double ne = av[i];
                        v = ne > 0.0 ? v / ne : 0.0;          // <eps> = sum(n eps) / sum(n)
                    } else if (ns > 0.0) {
                        v /= ns;
                    }
                    o[1 + (size_t)k * nn + i] = v;
                }
            break;
        }
        case PIC_DIAG_EEPF: {
            if (!need(8ull * (2 * kEepfBins + 2))) return PIC_EINVAL;
            std::vector<unsigned long long> h(2 * kEepfBins);
            ok = d2h(h.data(), ctx->d.eepf + (size_t)batch * 2 * kEepfBins, h.size() * 8);
            double* o = (double*)out;
            for (int i = 0; i < 2 * kEepfBins; ++i) o[i] = (double)h[i];
            o[2 * kEepfBins] = ctx->eepf_emax / kEepfBins;
            o[2 * kEepfBins + 1] = ds.eepf_samples;
            break;
        }
        case PIC_DIAG_RESET_AVG: {
            ok = hipMemset(ctx->d.avg + (size_t)batch * (S + 2) * nm, 0, 8ull * (S + 2) * nm) == hipSuccess;
            ok = ok && hipMemset(ctx->d.pavg + (size_t)batch * S * kPow * nm, 0, 8ull * S * kPow * nm) == hipSuccess;
            ok = ok && hipMemset(ctx->d.eepf + (size_t)batch * 2 * kEepfBins, 0, 8ull * 2 * kEepfBins) == hipSuccess;
            ok = ok && hipMemset(ctx->d.wedf + (size_t)batch * S * 2 * kEepfBins, 0, 8ull * S * 2 * kEepfBins) ==
                           hipSuccess;
            ds.avg_samples = 0.0;
            ds.eepf_samples = 0.0;
            ok = ok && hipMemcpy(ctx->d.diss + batch, &ds, sizeof(DisState), hipMemcpyHostToDevice) == hipSuccess;
            break;
        }
        case PIC_DIAG_CIRCUIT: {
            if (!need(16)) return PIC_EINVAL;
            double* o = (double*)out;
            ok = d2h(o, ctx->d.phi + (size_t)batch * nm, 8);
            const DisConst& dc = ctx->disc[batch];
            const bool circuit = dc.bc != PIC_BC_PERIODIC && dc.field_solve && dc.drive != PIC_DRIVE_VOLTAGE;
            o[1] = circuit && ds.circ_init
                       ? ds.qbase + source_charge(dc, (double)ds.step * dc.dt) + collected_charge(dc, cr.data(), S)
                       : 0.0;
            break;
        }
        case PIC_DIAG_GRAPHS: {
            if (!need(16)) return PIC_EINVAL;
            int64_t* o = (int64_t*)out;
            o[0] = ctx->graph_replays;
            o[1] = ctx->graph_steps;
            break;
        }
        case PIC_DIAG_RENEWED: {
            if (!need(8ull * S)) return PIC_EINVAL;
            int64_t* o = (int64_t*)out;
            for (int s = 0; s < S; ++s) o[s] = (int64_t)ev[(size_t)s * C_N + C_REN];
            break;
        }
        case PIC_DIAG_WALL_EDF: {
            const size_t nv = (size_t)S * 2 * kEepfBins;
            if (!need(8ull * (nv + S + 1))) return PIC_EINVAL;
            std::vector<unsigned long long> h(nv);
            ok = d2h(h.data(), ctx->d.wedf + (size_t)batch * nv, nv * 8);
            double* o = (double*)out;
            for (size_t i = 0; i < nv; ++i) o[i] = (double)h[i];
            for (int sp = 0; sp < S; ++sp) o[nv + sp] = ctx->wedf_emax[sp] / kEepfBins;
            o[nv + S] = ds.avg_samples;
            break;
        }
        case PIC_DIAG_WALL_ENERGY: {
            if (!need(8ull * 2 * S)) return PIC_EINVAL;
            std::vector<unsigned long long> we((size_t)S * 2);
            ok = d2h(we.data(), ctx->d.wen + (size_t)batch * S * 2, 8ull * 2 * S);
            const pic_config& c = ctx->cfg[batch];
            double* o = (double*)out;
            for (int sp = 0; sp < S; ++sp)
                for (int w = 0; w < 2; ++w)
                    o[2 * sp + w] = (double)we[2 * sp + w] / 1048576.0 * c.e_unit * c.species[sp].weight;
            break;
        }
        case PIC_DIAG_POWER: {
            if (!need(8ull * (1 + (size_t)kPow * S * nn))) return PIC_EINVAL;
            std::vector<double> pv((size_t)S * kPow * nm);
            ok = d2h(pv.data(), ctx->d.pavg + (size_t)batch * S * kPow * nm, pv.size() * 8);
            const double ns = ds.avg_samples;
            double* o = (double*)out;
            o[0] = ns;
            for (int sp = 0; sp < S; ++sp)
                for (int k = 0; k < kPow; ++k)
                    for (int i = 0; i < nn; ++i) {
                        const double v = pv[((size_t)sp * kPow + k) * nm + i];
                        o[1 + ((size_t)sp * kPow + k) * nn + i] = ns > 0.0 ? v / ns : 0.0;
                    }
            break;
        }
        case PIC_DIAG_TIMING: {
            if (!need(8ull * 6)) return PIC_EINVAL;
            prof_collect(ctx);
            double* o = (double*)out;
            o[0] = ctx->fin_n;
            o[1] = ctx->fin_ms;
            o[2] = ctx->push_n;
            o[3] = ctx->push_ms;
            o[4] = ctx->ev_n;
            o[5] = ctx->ev_ms;
            break;
        }
        case PIC_DIAG_CHARGE: {
            if (!need(16)) return PIC_EINVAL;
            std::vector<double> rho(nn);
            ok = d2h(rho.data(), ctx->d.rho + (size_t)batch * nm, 8ull * nn);
            const DisConst& dc = ctx->disc[batch];
            double q = 0.0;
            for (int i = 0; i < nn; ++i) {
                const double vol = (dc.bc != PIC_BC_PERIODIC && (i == 0 || i == nn - 1)) ? 0.5 * dc.dx : dc.dx;
                q += rho[i] * vol;
            }
            double qp = dc.rho_bg * dc.L;
            for (int s = 0; s < S; ++s) qp += ctx->segc[(size_t)batch * S + s].q * ctx->segc[(size_t)batch * S + s].w *
                                              (double)ss[s].live;
            ((double*)out)[0] = q;
            ((double*)out)[1] = qp;
            break;
        }
        default:
            return PIC_EINVAL;
    }
    if (!ok) return PIC_EHIP;
    return flags_status(ds.flags);
}

}  // extern "C"
