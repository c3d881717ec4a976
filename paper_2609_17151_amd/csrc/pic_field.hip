// Field side of the step: births appended after the last slot, the deposit
// turned into densities and charge, the 1D Poisson problem solved in FP64, the
// field at the nodes (paper Section 1: the field computed on a mesh from the
// particles' own charge; voltage waveform on the driven electrode), and the
// initial loading and leapfrog start.
//
// Poisson, -(phi[i-1] - 2 phi[i] + phi[i+1]) / dx^2 = rho[i] / eps0, is solved
// directly by two prefix sums.  With g = rho dx^2/eps0 and d[i] = phi[i+1]-phi[i]
// the equations read d[i] = d[0] - G[i], G[i] = g[1] + ... + g[i], so
// phi[i] = phi[0] + i d[0] - K[i] with K[i] = G[0] + ... + G[i-1]; the far
// boundary value fixes d[0] (Dirichlet: phi[N] = 0; periodic: phi[N] = phi[0]
// after removing the mean charge).  Both nested sums come out of one scan of
// (n, S, P) triples over contiguous runs of nodes, in a fixed order, in FP64.
#include "pic_device.h"
#include "pic_internal.h"
#include "pic_kernels.h"

namespace pic {

namespace {

constexpr int kFT = kFinThreads;          // finalize threads
constexpr int kWaves = kFT / 64;
constexpr int kBook = kFT - 64;           // first thread of the bookkeeping wave

// Prefix state of a run of nodes for the nested sums of the solve: n nodes,
// S = sum of g, P = sum over the run of the running sums of g, Q = sum over
// the run of the running sums of those (Q gives the sum of phi, hence the
// zero-mean gauge, without another reduction).  Appending run B after run A:
// n = nA + nB, S = SA + SB, P = PA + PB + nB SA,
// Q = QA + QB + nB PA + SA nB (nB + 1) / 2.  The all-zero run is the identity.
struct Run {
    double n, S, P, Q;
};

__device__ __forceinline__ Run run_combine(const Run& A, const Run& B)
{
    return Run{A.n + B.n, A.S + B.S, A.P + B.P + B.n * A.S,
               A.Q + B.Q + B.n * A.P + A.S * (0.5 * B.n * (B.n + 1.0))};
}

// DPP move of a double within a wave (zero where the source lane is invalid
// or the destination row is masked off)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffu), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void run_step(Run& v)
{
    Run o;
    o.n = dpp_f64<CTRL, ROW_MASK>(v.n);
    o.S = dpp_f64<CTRL, ROW_MASK>(v.S);
    o.P = dpp_f64<CTRL, ROW_MASK>(v.P);
    o.Q = dpp_f64<CTRL, ROW_MASK>(v.Q);
    v = run_combine(o, v);
}

// inclusive scan of Run over a wave, lanes in order: row shifts 1, 2, 4, 8
// within each row of 16 lanes, then the last lane of row 0 into rows 1 and 3
// and the last lane of row 1 into rows 2 and 3
__device__ __forceinline__ Run wave_run_scan(Run v)
{
    run_step<0x111, 0xf>(v);   // row_shr:1
    run_step<0x112, 0xf>(v);   // row_shr:2
    run_step<0x114, 0xf>(v);   // row_shr:4
    run_step<0x118, 0xf>(v);   // row_shr:8
    run_step<0x142, 0xa>(v);   // row_bcast:15
    run_step<0x143, 0xc>(v);   // row_bcast:31
    return v;
}

// sum over a wave in a fixed order (the same row shifts and broadcasts; the
// last lane ends with the total), returned to every lane.  The whole wave
// must be active.
__device__ __forceinline__ double wave_total_f64(double v)
{
    v += dpp_f64<0x111, 0xf>(v);
    v += dpp_f64<0x112, 0xf>(v);
    v += dpp_f64<0x114, 0xf>(v);
    v += dpp_f64<0x118, 0xf>(v);
    v += dpp_f64<0x142, 0xa>(v);
    v += dpp_f64<0x143, 0xc>(v);
    const unsigned long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffu), 63);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), 63);
    return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

}  // namespace

// A step that can have births takes two workgroups per discharge that run side
// by side: the first appends the step's births and then does the bookkeeping
// (counts, ids, kinetic-energy partial sums); the second, one node per thread
// (up to four), turns the deposit into densities and charge (and their
// per-wave sums, for the mean charge of a periodic mesh), solves for the field
// and adds the time averages.  The two share nothing of this step: the births'
// charge and diagnostics were deposited when they were staged.  Otherwise one
// workgroup does it all, its last wave the bookkeeping.  Poisson: every thread forms the run of its
// node, a wave-level scan and one scan over the waves' totals give K[i] and
// G[i] at every node, and phi follows directly; the totals also give the
// mean of phi.
__global__ __launch_bounds__(kFT) void finalize_kernel(FinArgs a)
{
    const DevPtrs& d = a.d;
    const bool split = a.mode == kFinStep && a.births_per_tile > 0;   // a births workgroup per discharge
    const bool births_wg = split && (blockIdx.x & 1u) == 0u;
    const int b = a.only_b >= 0 ? a.only_b : (int)(split ? blockIdx.x >> 1 : blockIdx.x);
    const int S = d.S, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const DisConst& dc = d.disc[b];
    DisState& ds = d.diss[b];
    const int nn = dc.n_nodes, nc = dc.n_cells;
    const int periodic = dc.bc == PIC_BC_PERIODIC;
    const size_t nb = (size_t)b * d.nodes_max;
    if (a.mode == kFinStep && blockIdx.x == 0 && threadIdx.x == 0) *d.tick += 1ull;
    if (a.mode == kFinStep && ds.retired) return;   // a retired discharge stays as it is

    __shared__ double s_a[kMaxCells + 1];     // rho, then phi
    __shared__ double s_bc[4];                // rho at the walls
    __shared__ double s_w[kWaves];
    __shared__ Run s_run[kWaves];

    // ---- births, appended after the last slot in the order of their tiles --
    // (and, inside a tile, of their parents): ionization electrons, then the
    // secondaries of each emitting ion species in turn; ionization ions in the
    // order of their electrons.  One pass per source segment: every thread
    // sums the birth counts of its run of consecutive tiles, a block scan of
    // those sums, then one birth per thread (its run found by a binary search
    // of the scan, its tile by a walk along the run), so the copies go out
    // together.
    // A tile's births are staged in any order; each carries its parent's
    // slot, and its rank among the tile's keys is its place.
    __shared__ int64_t s_app[kMaxSpecies], s_want[kMaxSpecies];
    __shared__ uint32_t s_scan[kWaves];
    __shared__ uint32_t s_tinc[kFT];         // inclusive prefix of the threads' runs' birth counts
    // the bookkeeping of a step, by one wave: counts, ids, kinetic energy
    auto bookkeeping = [&](bool births) {
        if (a.diag) {
            // kinetic-energy partials of the step's runs (zeros elsewhere),
            // fixed order, cleared after reading
            for (int s = 0; s < S; ++s) {
                SegState& st = d.segs[b * S + s];
                double* kpp = d.ke_part + st.tile_first;
                const int64_t ntl = st.ntiles;
                double acc_k = 0.0;
                for (int64_t t = lane; t < ntl; t += 64) {
                    acc_k += kpp[t];
                    kpp[t] = 0.0;
                }
                acc_k = wave_sum_f64(acc_k);
                if (lane == 0) st.ke = acc_k;
            }
        }
        if (lane < S) {                                 // one lane per species
            const int s = lane;
            SegState& st = d.segs[b * S + s];
            const int64_t app = births ? s_app[s] : 0, want = births ? s_want[s] : 0;
            if (app < want) {
                atomicOr(&ds.flags, kFlagCapacity);
                atomicAdd(&d.cnt[(((size_t)b * S + s) * kRep) * C_N + C_DROP], (unsigned long long)(want - app));
            }
            st.count += app;
            st.live += app - st.dead;
            st.dead = 0;
            st.staged = 0;
            st.next_id += (uint32_t)app;
            st.ntiles = 0;
        }
    };
    if (births_wg) {
        const SegState& s0 = d.segs[b * S + 0];
        const SegConst& c0 = d.segc[b * S + 0];
        const int64_t slot0 = s0.count, slot1 = S > 1 ? d.segs[b * S + 1].count : 0;
        const uint32_t id0 = s0.next_id, id1 = S > 1 ? d.segs[b * S + 1].next_id : 0u;
        const int io0 = s0.parity, io1 = S > 1 ? d.segs[b * S + 1].parity : 0;
        const int64_t cap0 = c0.cap, cap1 = S > 1 ? d.segc[b * S + 1].cap : 0;
        int64_t pos0 = slot0, pos1 = slot1;
        for (int src = 0; src < S; ++src) {
            const int g = b * S + src;
            if (src > 0 && !d.segc[g].emits) continue;
            if (d.segs[g].staged == 0) continue;          // no tile of this segment staged a birth
            const int64_t tf = d.segs[g].tile_first, nt = d.segs[g].ntiles;
            const bool pair = src == 0 && S > 1;            // ionization: an ion with every electron
            // thread tid covers the kt consecutive tiles from tid kt on (one
            // pass however many tiles the segment has)
            const int64_t kt = (nt + kFT - 1) / kFT;
            const uint32_t bpt = (uint32_t)a.births_per_tile;
            auto tile_births = [&](int64_t i) -> uint32_t {
                if (i >= nt) return 0u;
                const uint32_t bc = (uint32_t)d.bcnt[tf + i];
                return bc < bpt ? bc : bpt;               // more were counted as dropped
            };
            uint32_t c = 0;
            for (int64_t i = (int64_t)tid * kt; i < (int64_t)tid * kt + kt; ++i) c += tile_births(i);
            const uint32_t incl = wave_incl_scan_u32(c);
            if (lane == 63) s_scan[wid] = incl;
            __syncthreads();
            uint32_t wex = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                if (w < wid) wex += s_scan[w];
                tot += s_scan[w];
            }
            s_tinc[tid] = wex + incl;
            __syncthreads();
            for (uint32_t j = tid; j < tot; j += kFT) {
                // the thread holding birth j: the first with an inclusive
                // prefix above j; then the tile among its kt
                int lo = 0, hi = kFT - 1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_tinc[mid] > j) hi = mid; else lo = mid + 1;
                }
                uint32_t t0 = lo > 0 ? s_tinc[lo - 1] : 0u;
                int64_t ti = (int64_t)lo * kt;
                uint32_t nk = tile_births(ti);
                while (j - t0 >= nk) {
                    t0 += nk;
                    nk = tile_births(++ti);
                }
                const uint32_t k = j - t0;
                const Birth* tb = d.births + (size_t)(tf + ti) * a.births_per_tile;
                const Birth bb = tb[k];
                uint32_t rank = 0;
                for (uint32_t q = 0; q < nk; ++q) rank += tb[q].key < bb.key;
                const int64_t e = pos0 + t0 + rank;
                if (e < cap0) {
                    c0.cell[io0][e] = bb.cell;
                    c0.off[io0][e] = bb.off;
                    c0.vx[io0][e] = bb.vx;
                    c0.vy[io0][e] = bb.vy;
                    c0.vz[io0][e] = bb.vz;
                    c0.id[io0][e] = id0 + (uint32_t)(e - slot0);
                    if (c0.z[0]) c0.z[io0][e] = 0.0;
                }
                if (pair) {
                    const SegConst& c1 = d.segc[b * S + 1];
                    const int64_t q = pos1 + t0 + rank;
                    if (q < cap1) {
                        c1.cell[io1][q] = bb.cell;
                        c1.off[io1][q] = bb.off;
                        c1.vx[io1][q] = bb.ivx;
                        c1.vy[io1][q] = bb.ivy;
                        c1.vz[io1][q] = bb.ivz;
                        c1.id[io1][q] = id1 + (uint32_t)(q - slot1);
                        if (c1.z[0]) c1.z[io1][q] = 0.0;
                    }
                }
            }
            pos0 += tot;
            if (pair) pos1 += tot;
            __syncthreads();                              // s_scan and s_tinc are reused
        }
        if (tid == 0) {
            for (int s = 0; s < S; ++s) {
                s_want[s] = s == 0 ? pos0 - slot0 : (s == 1 ? pos1 - slot1 : 0);
                s_app[s] = 0;
            }
            s_app[0] = (pos0 < cap0 ? pos0 : cap0) - slot0;
            if (S > 1) s_app[1] = (pos1 < cap1 ? pos1 : cap1) - slot1;
        }
        __syncthreads();
        if (wid == 0) bookkeeping(true);
        return;
    }

    if (tid >= kBook) {
        if (lane == 0) s_w[wid] = 0.0;                  // no share of the charge sum
        if (a.mode == kFinStep && !split) bookkeeping(false);
    } else {
        // ---- densities and charge (into s_a) ------------------------------------
        double rsum = 0.0;
        for (int i = tid; i < nn; i += kBook) {
            double r;
            if (a.mode == kFinExternal) {
                r = a.rho_ext[i];
            } else {
                r = dc.rho_bg;
                const double wall = (!periodic && (i == 0 || i == nn - 1)) ? 2.0 : 1.0;
                for (int s = 0; s < S; ++s) {
                    unsigned long long* acc = d.acc + ((size_t)b * S + s) * kRep * d.nodes_max;
                    unsigned long long sum = 0ull;
#pragma unroll
                    for (int r = 0; r < kRep; ++r) {
                        sum += acc[(size_t)r * d.nodes_max + i];
                        acc[(size_t)r * d.nodes_max + i] = 0ull;
                    }
                    const double den = (double)sum * (dc.dens_coef[s] * wall);
                    d.dens[((size_t)b * S + s) * d.nodes_max + i] = den;
                    r += dc.q[s] * den;
                }
                d.rho[nb + i] = r;
            }
            s_a[i] = r;
            rsum += r;
        }
        if (periodic && dc.field_solve) {               // the waves' shares of the total charge
            const double w = wave_total_f64(rsum);
            if (lane == 0) s_w[wid] = w;
        }
    }
    __syncthreads();

    // ---- Poisson: phi[i] = phi0 + i d0 - K[i] (file header) -------------------
    const double t = a.mode == kFinExternal ? a.t_ext
                   : (double)(ds.step + (a.mode == kFinStep ? 1 : 0)) * dc.dt;
    double circ_qbase = 0.0;                  // circuit: the conductor's base charge of this solve
    bool win_closed = false;                  // an RF window ended with this step
    if (!periodic && tid == 0) {
        s_bc[0] = s_a[0];
        s_bc[1] = s_a[nn - 1];
    }
    if (dc.field_solve) {
        double mean = 0.0;
        if (periodic) {
            double tot = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) tot += s_w[w];
            mean = tot / nn;
        }
        // thread tid holds the consecutive nodes kNodesPerThread tid + j; only
        // the waves that hold nodes take part (one per SIMD on meshes of up to
        // 1024 nodes), each thread summing its own nodes in sequence
        const double c2 = dc.c2;
        const int i0 = tid * kNodesPerThread;
        const bool active = wid * 64 * kNodesPerThread < nn;     // uniform over the wave
        double g[kNodesPerThread];
        Run inc{0.0, 0.0, 0.0, 0.0};
        if (active) {
            Run loc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int j = 0; j < kNodesPerThread; ++j) {
                const int i = i0 + j;
                g[j] = 0.0;
                if (i < nn) {
                    const bool unknown = i >= 1 && (periodic ? i < nn : i < nn - 1);
                    g[j] = unknown ? (s_a[i] - mean) * c2 : 0.0;
                    loc.n += 1.0;                          // one node appended
                    loc.S += g[j];
                    loc.P += loc.S;
                    loc.Q += loc.P;
                }
            }
            inc = wave_run_scan(loc);
            if (lane == 63) s_run[wid] = inc;
        }
        __syncthreads();
        // inclusive prefix over the waves, in place (the wave's reads are
        // issued before its writes); waves without nodes count as empty runs
        if (tid < 64) {
            const Run v = (tid < kWaves && tid * 64 * kNodesPerThread < nn) ? s_run[tid] : Run{0.0, 0.0, 0.0, 0.0};
            const Run vi = wave_run_scan(v);
            if (tid < kWaves) s_run[tid] = vi;
        }
        __syncthreads();
        const Run all = s_run[kWaves - 1];
        const double totS = all.S, totP = all.P;
        double phi0, d0;
        if (periodic) {
            phi0 = 0.0;
            d0 = totP / nc;                              // H = sum_{i<N} G[i]
        } else if (dc.drive == PIC_DRIVE_VOLTAGE) {
            phi0 = source_voltage(dc, t);
            d0 = (totP - totS - phi0) / nc;              // H = P - G[N], phi[N] = 0
        } else {
            // external circuit: psi (phi0 = 0) has phi[1] = (P - G[N]) / N; its
            // surface field at x = 0 by Gauss's law over the half cell; then
            // q = eps0 (E0[psi] + phi0 / L) + C (phi0 - V) gives phi0
            const double e0psi = -((totP - totS) / nc) * dc.inv_dx - s_bc[0] * dc.wall_coef;
            const bool capd = dc.drive == PIC_DRIVE_CAPACITOR;
            const double C = capd ? dc.cap : 0.0;
            const double v = capd ? source_voltage(dc, t) : 0.0;
            const double qc = collected_charge(dc, d.cnt + (size_t)b * S * kRep * C_N, S);
            const double qs = source_charge(dc, t);
            // first solve: the electrode starts at the source's potential
            const double qb = ds.circ_init ? ds.qbase : dc.eps0 * (v / dc.L + e0psi) - qs - qc;
            phi0 = (C * v + (qb + qs + qc) - dc.eps0 * e0psi) / (C + dc.eps0 / dc.L);
            d0 = (totP - totS - phi0) / nc;
            circ_qbase = qb;
        }
        // zero-mean gauge of a periodic mesh: the sum of phi[i] is
        // d0 N (N - 1) / 2 minus the sum of K[i], and the K[i] = P_incl[i] - G[i]
        // sum to Q - P over all nodes
        const double pm = periodic ? (d0 * (0.5 * (double)nn * (double)(nn - 1)) - (all.Q - all.P)) / nn : 0.0;
        if (active) {
            // the runs before this thread: the waves before, then the lanes before
            Run lx;
            lx.n = __shfl_up(inc.n, 1, 64);
            lx.S = __shfl_up(inc.S, 1, 64);
            lx.P = __shfl_up(inc.P, 1, 64);
            lx.Q = 0.0;
            if (lane == 0) lx = Run{0.0, 0.0, 0.0, 0.0};
            const Run ex = wid > 0 ? run_combine(s_run[wid - 1], lx) : lx;
            // every read of rho was before the barrier after the wave scans
            double G = ex.S, P = ex.P;
#pragma unroll
            for (int j = 0; j < kNodesPerThread; ++j) {
                const int i = i0 + j;
                if (i >= nn) break;
                G += g[j];
                P += G;                                    // K[i] = P - G[i]
                double ph = phi0 + (double)i * d0 - (P - G);
                if (!periodic && i == nn - 1) ph = 0.0;
                if (i == 0) ph = phi0;
                s_a[i] = ph - pm;
            }
        }
    } else {
        __syncthreads();                                 // the wall charges are read
        for (int i = tid; i < nn; i += kFT) s_a[i] = 0.0;
    }
    __syncthreads();

    // ---- field at the nodes (all threads) ------------------------------------
    auto efield = [&](int i) -> double {
        if (!dc.field_solve) return 0.0;
        if (periodic) {
            const int im = i == 0 ? nn - 1 : i - 1, ip = i == nn - 1 ? 0 : i + 1;
            return (s_a[im] - s_a[ip]) * dc.inv_2dx;
        }
        if (i == 0) return -(s_a[1] - s_a[0]) * dc.inv_dx - s_bc[0] * dc.wall_coef;
        if (i == nn - 1) return -(s_a[nn - 1] - s_a[nn - 2]) * dc.inv_dx + s_bc[1] * dc.wall_coef;
        return (s_a[i - 1] - s_a[i + 1]) * dc.inv_2dx;
    };
    double fe_loc = 0.0;
    for (int i = tid; i < nn; i += kFT) {
        const double e = efield(i);
        const double vol = (!periodic && (i == 0 || i == nn - 1)) ? 0.5 : 1.0;
        fe_loc += e * e * vol;
        if (a.mode == kFinExternal) {
            if (a.phi_out) a.phi_out[i] = s_a[i];
            if (a.e_out) a.e_out[i] = e;
        } else {
            d.phi[nb + i] = s_a[i];
            d.ef[nb + i] = e;
        }
    }
    if (a.mode == kFinExternal) return;
    for (int c = tid; c < nc; c += kFT) {
        const int c1 = (periodic && c + 1 == nc) ? 0 : c + 1;
        d.epair[(size_t)b * d.cells_max + c] = make_float2((float)efield(c), (float)efield(c1));
    }
    // field energy: per-wave sums, added in wave order
    fe_loc = wave_total_f64(fe_loc);
    if (lane == 0) s_w[wid] = fe_loc;

    // ---- time averages -------------------------------------------------------
    if (a.mode == kFinStep && a.diag) {
        double* av = d.avg + (size_t)b * (S + 2) * d.nodes_max;
        unsigned long long* ea = d.eacc + nb;
        const double ecoef = dc.dens_coef[0] * kDepScale / 1048576.0;   // w / dx / 2^20
        for (int i = tid; i < nn; i += kFT) {
            for (int s = 0; s < S; ++s)
                av[(size_t)s * d.nodes_max + i] += d.dens[((size_t)b * S + s) * d.nodes_max + i];
            av[(size_t)S * d.nodes_max + i] += s_a[i];
            const double wall = (!periodic && (i == 0 || i == nn - 1)) ? 2.0 : 1.0;
            av[(size_t)(S + 1) * d.nodes_max + i] += (double)ea[i] * ecoef * wall;   // n_e <eps>
            ea[i] = 0ull;
        }
        // flux, momentum flux and the power the new field gives each species,
        // and the power decomposition of the electron (and ion) momentum
        // balance, m dGamma/dt + d(m n <vx^2>)/dx = q n E + R, multiplied by
        // u = Gamma / n: inertia u (m dGamma/dt + d(m Gamma^2 / n)/dx),
        // pressure u dp/dx with p = m (n <vx^2> - Gamma^2 / n), and the ohmic
        // part q Gamma E - inertia - pressure (formed by the reader).  The time
        // derivative uses the flux of the previous step when that step was
        // sampled; gradients are central inside, one-sided at a wall node.
        const bool prev = ds.pw_next == ds.step;
        double* kt = d.ptmp + (size_t)b * 2 * d.nodes_max;    // m Gamma^2 / n and p at the nodes
        double* pt = kt + d.nodes_max;
        for (int s = 0; s < S; ++s) {
            unsigned long long* ma = d.macc + ((size_t)b * S + s) * 2 * d.nodes_max;
            double* pv = d.pavg + ((size_t)b * S + s) * kPow * d.nodes_max;
            const double* dn = d.dens + ((size_t)b * S + s) * d.nodes_max;
            double* gp = d.gprev + ((size_t)b * S + s) * d.nodes_max;
            const double m = dc.mass[s];
            __syncthreads();                             // the previous species' gradients are read
            for (int i = tid; i < nn; i += kFT) {
                const double wall = (!periodic && (i == 0 || i == nn - 1)) ? 2.0 : 1.0;
                const double G = (double)(long long)ma[i] * dc.flux_coef[s] * wall;
                const double M = (double)(long long)ma[d.nodes_max + i] * dc.mom_coef[s] * wall;
                const double nd = dn[i];
                const double K = nd > 0.0 ? m * G * G / nd : 0.0;
                kt[i] = K;
                pt[i] = m * M - K;
            }
            __threadfence_block();
            __syncthreads();
            for (int i = tid; i < nn; i += kFT) {
                const double wall = (!periodic && (i == 0 || i == nn - 1)) ? 2.0 : 1.0;
                const double G = (double)(long long)ma[i] * dc.flux_coef[s] * wall;
                const double M = (double)(long long)ma[d.nodes_max + i] * dc.mom_coef[s] * wall;
                ma[i] = 0ull;
                ma[d.nodes_max + i] = 0ull;
                const double e = efield(i) + dc.e_ext[0];   // the mesh field and the imposed one
                const double nd = dn[i];
                const double u = nd > 0.0 ? G / nd : 0.0;
                int il, ir;
                double h;
                if (periodic) {
                    il = i == 0 ? nn - 1 : i - 1;
                    ir = i == nn - 1 ? 0 : i + 1;
                    h = 2.0 * dc.dx;
                } else {
                    il = i > 0 ? i - 1 : i;
                    ir = i < nn - 1 ? i + 1 : i;
                    h = (double)(ir - il) * dc.dx;
                }
                const double dk = (kt[ir] - kt[il]) / h, dp = (pt[ir] - pt[il]) / h;
                const double dgdt = prev ? (G - gp[i]) / dc.dt : 0.0;
                pv[i] += G;
                pv[(size_t)d.nodes_max + i] += M;
                pv[2 * (size_t)d.nodes_max + i] += dc.q[s] * G * e;
                pv[3 * (size_t)d.nodes_max + i] += u * (m * dgdt + dk);
                pv[4 * (size_t)d.nodes_max + i] += u * dp;
                gp[i] = G;
            }
        }
        // an RF window ends with this step: its sums go to the ring (each
        // thread its own nodes, as above) and the accumulators restart
        if (ds.win_len > 0 && (ds.step + 1 - ds.win_start) % ds.win_len == 0) {
            const size_t stride = 1 + (size_t)(S + 2) * d.nodes_max;
            double* w = d.wring + ((size_t)b * kWindowRing + (size_t)(ds.nwin % kWindowRing)) * stride;
            for (int i = tid; i < nn; i += kFT)
                for (int k = 0; k < S + 2; ++k) {
                    w[1 + (size_t)k * d.nodes_max + i] = av[(size_t)k * d.nodes_max + i];
                    av[(size_t)k * d.nodes_max + i] = 0.0;
                }
            if (tid == 0) w[0] = ds.avg_samples + 1.0;   // this step's sample included
            win_closed = true;
        }
    }
    __syncthreads();
    if (tid == 0) {
        double fe = 0.0;
        for (int w = 0; w < kWaves; ++w) fe += s_w[w];
        ds.fe = 0.5 * dc.eps0 * dc.dx * fe;
        if (!periodic && dc.field_solve && dc.drive != PIC_DRIVE_VOLTAGE && !ds.circ_init) {
            ds.qbase = circ_qbase;
            ds.circ_init = 1;
        }
        if (a.mode == kFinStep) {
            if (a.diag) {
                ds.pw_next = ds.step + 1;                // this step's flux is stored
                ds.avg_samples += 1.0;
                ds.eepf_samples += 1.0;
                if (win_closed) {
                    ds.avg_samples = 0.0;
                    ds.nwin += 1;
                }
            }
            ds.step += 1;
        }
    }
}

hipError_t launch_finalize(const FinArgs& a, hipStream_t st)
{
    const unsigned per = (a.mode == kFinStep && a.births_per_tile > 0) ? 2u : 1u;   // births workgroup
    const unsigned g = (a.only_b >= 0 ? 1u : (unsigned)a.d.B) * per;
    hipLaunchKernelGGL(finalize_kernel, dim3(g), dim3(kFT), 0, st, a);
    return hipGetLastError();
}

// ---- loading: one thread per particle, FP64 --------------------------------
__global__ __launch_bounds__(256) void load_kernel(LoadArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const DevPtrs& d = a.d;
    const DisConst& dc = d.disc[a.b];
    const SegConst& sc = d.segc[a.b * d.S + a.s];
    const double L = dc.L;
    const uint4 r0 = philox10((uint32_t)j, 0xFFFFFFFFu, ((uint32_t)a.s << 24) | 0u, 0u,
                              dc.key0, dc.key1);
    const uint4 r1 = philox10((uint32_t)j, 0xFFFFFFFFu, ((uint32_t)a.s << 24) | 1u, 0u,
                              dc.key0, dc.key1);
    const double u = u01d(r0.x);
    const double x0 = a.load == PIC_LOAD_STRATIFIED ? ((double)j + u) * L / (double)a.n : u * L;
    double x = x0;
    if (a.perturb_eps != 0.0 && a.perturb_mode != 0) {
        const double kw = 6.283185307179586476925286766559 * a.perturb_mode / L;
        const double ep = a.perturb_eps;
        for (int it = 0; it < 60; ++it) {
            const double fx = x + ep / kw * sin(kw * x) - x0;
            const double dd = fx / (1.0 + ep * cos(kw * x));
            x -= dd;
            if (fabs(dd) <= 1e-15 * L) break;
        }
    }
    if (x < 0.0) x += L;
    if (x >= L) x -= L;
    const double xi = x / dc.dx;
    int c = (int)floor(xi);
    float f = (float)(xi - (double)c);
    if (f >= 1.0f) {
        f -= 1.0f;
        c += 1;
    }
    if (c >= dc.n_cells) {
        if (dc.bc == PIC_BC_PERIODIC) c -= dc.n_cells;
        else { c = dc.n_cells - 1; f = 0x1.fffffep-1f; }
    }
    double g0, g1, g2, g3;
    box_muller_d(u01d(r1.x), u01d(r1.y), g0, g1);
    box_muller_d(u01d(r1.z), u01d(r1.w), g2, g3);
    const int p = d.segs[a.b * d.S + a.s].parity;
    sc.cell[p][j] = c;
    sc.off[p][j] = f;
    sc.vx[p][j] = (float)(a.drift[0] + a.vth * g0);
    sc.vy[p][j] = (float)(a.drift[1] + a.vth * g1);
    sc.vz[p][j] = (float)(a.drift[2] + a.vth * g2);
    sc.id[p][j] = (uint32_t)j;
}

// Start from profiles: density and temperature at m points evenly spread over
// [0, L], linear in between.  x_j = F^-1((j + u_j) / n) with F the integral of
// the density; inside piece k the integral from x_k is h (n_k t + dn t^2 / 2)
// at x = x_k + t h, so t is the root 2q / (n_k + sqrt(n_k^2 + 2 dn q)) of
// (dn / 2) t^2 + n_k t = q (this form holds for dn = 0 and dn < 0 too).
// Velocities: three Box-Muller normals times sqrt(e T(x_j) / m).  Draws as in
// the plain load, so a uniform profile gives the stratified positions.
__global__ __launch_bounds__(256) void profile_load_kernel(ProfileArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const DevPtrs& d = a.d;
    const DisConst& dc = d.disc[a.b];
    const SegConst& sc = d.segc[a.b * d.S + a.s];
    const double L = dc.L, h = L / (double)(a.m - 1);
    const uint4 r0 = philox10((uint32_t)j, 0xFFFFFFFFu, ((uint32_t)a.s << 24) | 0u, 0u, dc.key0, dc.key1);
    const uint4 r1 = philox10((uint32_t)j, 0xFFFFFFFFu, ((uint32_t)a.s << 24) | 1u, 0u, dc.key0, dc.key1);
    const double y = ((double)j + u01d(r0.x)) / (double)a.n * a.cum[a.m - 1];
    int lo = 0, hi = a.m - 1;                 // last piece k with cum[k] <= y
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.cum[mid] <= y) lo = mid; else hi = mid;
    }
    const int k = lo;
    const double nk = a.dens[k], dn = a.dens[k + 1] - nk;
    const double q = (y - a.cum[k]) / h;
    double t = 0.0;
    if (q > 0.0) {
        const double den = nk + sqrt(fmax(nk * nk + 2.0 * dn * q, 0.0));
        t = den > 0.0 ? 2.0 * q / den : 1.0;
    }
    t = fmin(fmax(t, 0.0), 1.0);
    double x = ((double)k + t) * h;
    if (x >= L) x = L * (1.0 - 1e-16);
    const double xi = x / dc.dx;
    int c = (int)floor(xi);
    float f = (float)(xi - (double)c);
    if (f >= 1.0f) {
        f -= 1.0f;
        c += 1;
    }
    if (c >= dc.n_cells) {
        c = dc.n_cells - 1;
        f = 0x1.fffffep-1f;
    }
    const double T = a.temp[k] + t * (a.temp[k + 1] - a.temp[k]);
    const double vth = sqrt(a.e_over_m * fmax(T, 0.0));
    double g0, g1, g2, g3;
    box_muller_d(u01d(r1.x), u01d(r1.y), g0, g1);
    box_muller_d(u01d(r1.z), u01d(r1.w), g2, g3);
    const int p = d.segs[a.b * d.S + a.s].parity;
    sc.cell[p][j] = c;
    sc.off[p][j] = f;
    sc.vx[p][j] = (float)(vth * g0);
    sc.vy[p][j] = (float)(vth * g1);
    sc.vz[p][j] = (float)(vth * g2);
    sc.id[p][j] = (uint32_t)j;
}

hipError_t launch_profile_load(const ProfileArgs& a, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(profile_load_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_load(const LoadArgs& a, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    const unsigned g = (unsigned)((a.n + 255) / 256);
    hipLaunchKernelGGL(load_kernel, dim3(g), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ---- deposit only (start, restart) ------------------------------------------
__global__ __launch_bounds__(256) void deposit_kernel(DevPtrs d, int only_b)
{
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long* hist = reinterpret_cast<unsigned long long*>(smem);
    const int s = blockIdx.y;
    const int b = only_b >= 0 ? only_b : (int)blockIdx.z;
    const SegConst& sc = d.segc[b * d.S + s];
    const SegState& st = d.segs[b * d.S + s];
    const DisConst& dc = d.disc[b];
    const int nn = dc.n_nodes, nc = dc.n_cells, periodic = dc.bc == PIC_BC_PERIODIC;
    const int64_t base = (int64_t)blockIdx.x * 1024;
    if (base >= st.count) return;
    for (int i = threadIdx.x; i < nn; i += 256) hist[i] = 0ull;
    __syncthreads();
    const int p = st.parity;
    for (int j = 0; j < 4; ++j) {
        const int64_t k = base + j * 256 + threadIdx.x;
        if (k >= st.count) break;
        int c = sc.cell[p][k];
        const float f = sc.off[p][k];
        if ((unsigned)c >= (unsigned)nc) {
            atomicOr(&d.diss[b].flags, kFlagCell);
            continue;
        }
        uint32_t q = (uint32_t)(f * 4294967296.0f);
        if (f >= 1.0f) q = 0xFFFFFFFFu;
        const int c1 = (periodic && c + 1 == nc) ? 0 : c + 1;
        atomicAdd(&hist[c], (unsigned long long)(0x100000000ull - q));
        atomicAdd(&hist[c1], (unsigned long long)q);
    }
    __syncthreads();
    unsigned long long* acc = d.acc + (((size_t)b * d.S + s) * kRep + blockIdx.x % kRep) * d.nodes_max;
    for (int i = threadIdx.x; i < nn; i += 256) {
        const unsigned long long v = hist[i];
        if (v) atomicAdd(&acc[i], v);
    }
}

hipError_t launch_deposit(const DevPtrs& d, int only_b, int64_t max_count, hipStream_t st)
{
    if (max_count <= 0) return hipSuccess;
    const dim3 g((unsigned)((max_count + 1023) / 1024), (unsigned)d.S, only_b >= 0 ? 1u : (unsigned)d.B);
    hipLaunchKernelGGL(deposit_kernel, g, dim3(256), (size_t)d.nodes_max * 8, st, d, only_b);
    return hipGetLastError();
}

// ---- leapfrog start: v^{-1/2} = Boris(v^0; E^0, B, -dt/2), FP64 ------------------
__global__ __launch_bounds__(256) void halfstep_kernel(DevPtrs d, int only_b)
{
    const int s = blockIdx.y;
    const int b = only_b >= 0 ? only_b : (int)blockIdx.z;
    const SegConst& sc = d.segc[b * d.S + s];
    const SegState& st = d.segs[b * d.S + s];
    const DisConst& dc = d.disc[b];
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= st.count) return;
    const int p = st.parity;
    const int c = sc.cell[p][k];
    const double f = sc.off[p][k];
    const int nc = dc.n_cells;
    const int c1 = (dc.bc == PIC_BC_PERIODIC && c + 1 == nc) ? 0 : c + 1;
    const double* ef = d.ef + (size_t)b * d.nodes_max;
    const double h = -0.5 * dc.dt;
    const double qm = sc.qm;
    const double aa = 0.5 * qm * h;
    const double e0 = (1.0 - f) * ef[c] + f * ef[c1] + dc.e_ext[0];
    const double e1 = dc.e_ext[1], e2 = dc.e_ext[2];
    const double bx = dc.b_ext[0], by = dc.b_ext[1], bz = dc.b_ext[2];
    double vx = (double)sc.vx[p][k] + aa * e0, vy = (double)sc.vy[p][k] + aa * e1,
           vz = (double)sc.vz[p][k] + aa * e2;
    const double tx = aa * bx, ty = aa * by, tz = aa * bz;
    const double t2 = tx * tx + ty * ty + tz * tz, sf = 2.0 / (1.0 + t2);
    const double px = vx + (vy * tz - vz * ty), py = vy + (vz * tx - vx * tz), pz = vz + (vx * ty - vy * tx);
    vx += sf * (py * tz - pz * ty);
    vy += sf * (pz * tx - px * tz);
    vz += sf * (px * ty - py * tx);
    sc.vx[p][k] = (float)(vx + aa * e0);
    sc.vy[p][k] = (float)(vy + aa * e1);
    sc.vz[p][k] = (float)(vz + aa * e2);
}

hipError_t launch_halfstep(const DevPtrs& d, int only_b, int64_t max_count, hipStream_t st)
{
    if (max_count <= 0) return hipSuccess;
    const dim3 g((unsigned)((max_count + 255) / 256), (unsigned)d.S, only_b >= 0 ? 1u : (unsigned)d.B);
    hipLaunchKernelGGL(halfstep_kernel, g, dim3(256), 0, st, d, only_b);
    return hipGetLastError();
}

}  // namespace pic
