// Field side of the step: births appended after the survivors, the deposit
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
// after removing the mean charge).  One 1024-thread workgroup per discharge,
// four nodes per thread, FP64 scans in a fixed order.
#include "pic_device.h"
#include "pic_internal.h"
#include "pic_kernels.h"

namespace pic {

namespace {

__device__ double block_excl_scan(double v, double* s_w, double& total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const double incl = wave_incl_scan_f64(v);
    if (lane == 63) s_w[wid] = incl;
    __syncthreads();
    double off = 0.0, tot = 0.0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) {
        if (w < wid) off += s_w[w];
        tot += s_w[w];
    }
    __syncthreads();
    total = tot;
    return off + incl - v;
}

__device__ double block_sum(double v, double* s_w)
{
    double tot;
    (void)block_excl_scan(v, s_w, tot);
    return tot;
}

}  // namespace

__global__ __launch_bounds__(kFinThreads) void finalize_kernel(FinArgs a)
{
    constexpr int P = kNodesPerThread;
    const DevPtrs& d = a.d;
    const int b = a.only_b >= 0 ? a.only_b : (int)blockIdx.x;
    const int S = d.S, tid = threadIdx.x;
    const DisConst& dc = d.disc[b];
    DisState& ds = d.diss[b];
    const int nn = dc.n_nodes, nc = dc.n_cells;
    const int periodic = dc.bc == PIC_BC_PERIODIC;
    const size_t nb = (size_t)b * d.nodes_max;

    __shared__ double s_w[kFinThreads / 64];
    __shared__ double s_phi[kMaxCells + 1];   // phi, then E
    __shared__ double s_bcast[4];

    // ---- births after the survivors; counts, ids and copies ---------------
    if (a.mode == kFinStep) {
        const int64_t n_ion = d.segs[b * S + 0].births;
        const int64_t n_see = S > 1 ? d.segs[b * S + 1].see_births : 0;
        for (int s = 0; s < S; ++s) {
            const SegConst& sc = d.segc[b * S + s];
            SegState& st = d.segs[b * S + s];
            const int64_t surv = st.surv;
            const int64_t nbirth = s == 0 ? n_ion + n_see : (s == 1 ? n_ion : 0);
            int64_t nmove = nbirth;
            if (nmove > sc.bcap) nmove = sc.bcap;
            if (nmove > sc.cap - surv) nmove = sc.cap - surv;
            const int out = sc.compacts ? (st.parity ^ 1) : st.parity;
            for (int64_t k = tid; k < nmove; k += kFinThreads) {
                sc.cell[out][surv + k] = sc.bcell[k];
                sc.off[out][surv + k] = sc.boff[k];
                sc.vx[out][surv + k] = sc.bvx[k];
                sc.vy[out][surv + k] = sc.bvy[k];
                sc.vz[out][surv + k] = sc.bvz[k];
                sc.id[out][surv + k] = sc.bid[k];
            }
            // kinetic energy of the step, tiles summed in a fixed order
            double kp = 0.0;
            for (int64_t t = tid; t < st.ntiles; t += kFinThreads)
                kp += d.ke_part[(size_t)s * d.tiles_max + st.tile_first + t];
            const double ke = block_sum(kp, s_w);
            __syncthreads();
            if (tid == 0) {
                if (nmove < nbirth) {
                    atomicOr(&ds.flags, kFlagCapacity);
                    st.dropped += (unsigned long long)(nbirth - nmove);
                }
                st.count = surv + nmove;
                st.next_id += (uint32_t)nmove;
                st.parity = out;
                st.ke = ke;
            }
            __syncthreads();
        }
        __syncthreads();
        if (tid == 0) {
            for (int s = 0; s < S; ++s) {
                SegState& st = d.segs[b * S + s];
                st.births = 0;
                st.see_births = 0;
                st.surv = st.count;
                st.ntiles = 0;
            }
        }
    }

    // ---- densities and charge ---------------------------------------------
    double rho[P];
    const double dx = dc.dx;
#pragma unroll
    for (int j = 0; j < P; ++j) rho[j] = 0.0;
    if (a.mode == kFinExternal) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int i = tid * P + j;
            if (i < nn) rho[j] = a.rho_ext[i];
        }
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int i = tid * P + j;
            if (i < nn) rho[j] = dc.rho_bg;
        }
        for (int s = 0; s < S; ++s) {
            const SegConst& sc = d.segc[b * S + s];
            unsigned long long* acc = d.acc + ((size_t)b * S + s) * d.nodes_max;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const int i = tid * P + j;
                if (i >= nn) continue;
                const double sum = (double)acc[i] * (1.0 / kDepScale);
                acc[i] = 0ull;
                const double vol = (!periodic && (i == 0 || i == nn - 1)) ? 0.5 * dx : dx;
                const double den = sc.w * sum / vol;
                d.dens[((size_t)b * S + s) * d.nodes_max + i] = den;
                rho[j] += sc.q * den;
            }
        }
    }

    // ---- Poisson -------------------------------------------------------------
    double phi[P];
    const double t = a.mode == kFinExternal ? a.t_ext
                   : (double)(ds.step + (a.mode == kFinStep ? 1 : 0)) * dc.dt;
    if (!dc.field_solve) {
#pragma unroll
        for (int j = 0; j < P; ++j) phi[j] = 0.0;
    } else {
        const double c2 = dx * dx / dc.eps0;
        double mean = 0.0;
        if (periodic) {
            double loc = 0.0;
#pragma unroll
            for (int j = 0; j < P; ++j) loc += rho[j];
            mean = block_sum(loc, s_w) / nn;
        }
        double g[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int i = tid * P + j;
            g[j] = 0.0;
            if (i >= 1 && (periodic ? i < nn : i < nn - 1)) g[j] = (rho[j] - mean) * c2;
        }
        // G = inclusive prefix of g
        double G[P], run = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            run += g[j];
            G[j] = run;
        }
        double totg;
        const double offg = block_excl_scan(run, s_w, totg);
#pragma unroll
        for (int j = 0; j < P; ++j) G[j] += offg;
        // K = exclusive prefix of G
        double K[P], runk = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int i = tid * P + j;
            K[j] = runk;
            if (i < nn) runk += G[j];
        }
        double totG;
        const double offk = block_excl_scan(runk, s_w, totG);
#pragma unroll
        for (int j = 0; j < P; ++j) K[j] += offk;
        double phi0, d0;
        const int N = nc;
        if (periodic) {
            phi0 = 0.0;
            d0 = totG / N;                       // H = sum_{i<N} G[i]
        } else {
            phi0 = dc.v_amp * sin(6.283185307179586476925286766559 * dc.v_freq * t + dc.v_phase);
            // H = K[N] = sum_{i<N} G[i] = totG - G[N]
            if (tid * P <= N && N < tid * P + P) s_bcast[0] = G[N - tid * P];
            __syncthreads();
            const double H = totG - s_bcast[0];
            d0 = (0.0 - phi0 + H) / N;
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int i = tid * P + j;
            phi[j] = phi0 + (double)i * d0 - K[j];
        }
        if (!periodic) {
            if (tid * P <= N && N < tid * P + P) phi[N - tid * P] = 0.0;
            if (tid == 0) phi[0] = phi0;
        } else {
            double loc = 0.0;
#pragma unroll
            for (int j = 0; j < P; ++j)
                if (tid * P + j < nn) loc += phi[j];
            const double pm = block_sum(loc, s_w) / nn;
#pragma unroll
            for (int j = 0; j < P; ++j) phi[j] -= pm;
        }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int i = tid * P + j;
        if (i < nn) s_phi[i] = phi[j];
    }
    // wall charge for Gauss's law at the electrodes
    if (!periodic) {
        if (tid == 0) s_bcast[1] = rho[0];
        if (tid * P <= nn - 1 && nn - 1 < tid * P + P) s_bcast[2] = rho[nn - 1 - tid * P];
    }
    __syncthreads();

    // ---- field at the nodes ----------------------------------------------------
    double ef[P];
    double fe_loc = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int i = tid * P + j;
        ef[j] = 0.0;
        if (i >= nn || !dc.field_solve) continue;
        if (periodic) {
            const int im = i == 0 ? nn - 1 : i - 1, ip = i == nn - 1 ? 0 : i + 1;
            ef[j] = (s_phi[im] - s_phi[ip]) / (2.0 * dx);
        } else if (i == 0) {
            ef[j] = -(s_phi[1] - s_phi[0]) / dx - s_bcast[1] * dx / (2.0 * dc.eps0);
        } else if (i == nn - 1) {
            ef[j] = -(s_phi[nn - 1] - s_phi[nn - 2]) / dx + s_bcast[2] * dx / (2.0 * dc.eps0);
        } else {
            ef[j] = (s_phi[i - 1] - s_phi[i + 1]) / (2.0 * dx);
        }
    }
    if (a.mode == kFinExternal) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int i = tid * P + j;
            if (i < nn) {
                if (a.phi_out) a.phi_out[i] = phi[j];
                if (a.e_out) a.e_out[i] = ef[j];
            }
        }
        return;
    }
    __syncthreads();                     // every thread has read s_phi
    double* s_ef = s_phi;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int i = tid * P + j;
        if (i >= nn) continue;
        d.rho[nb + i] = rho[j];
        d.phi[nb + i] = phi[j];
        d.ef[nb + i] = ef[j];
        s_ef[i] = ef[j];
        const double vol = (!periodic && (i == 0 || i == nn - 1)) ? 0.5 * dx : dx;
        fe_loc += ef[j] * ef[j] * vol;
    }
    const double fe = 0.5 * dc.eps0 * block_sum(fe_loc, s_w);
    // block_sum synchronised the block, so s_ef is complete
    for (int c = tid; c < nc; c += kFinThreads) {
        const int c1 = (periodic && c + 1 == nc) ? 0 : c + 1;
        d.epair[(size_t)b * d.cells_max + c] = make_float2((float)s_ef[c], (float)s_ef[c1]);
    }

    // ---- time averages -------------------------------------------------------
    if (a.mode == kFinStep && a.diag) {
        double* av = d.avg + (size_t)b * (S + 2) * d.nodes_max;
        unsigned long long* ea = d.eacc + nb;
        for (int i = tid; i < nn; i += kFinThreads) {
            for (int s = 0; s < S; ++s)
                av[(size_t)s * d.nodes_max + i] += d.dens[((size_t)b * S + s) * d.nodes_max + i];
            av[(size_t)S * d.nodes_max + i] += d.phi[nb + i];
            const double vol = (!periodic && (i == 0 || i == nn - 1)) ? 0.5 * dx : dx;
            const double esum = (double)ea[i] * (1.0 / 1048576.0);   // eV x weight fraction
            ea[i] = 0ull;
            av[(size_t)(S + 1) * d.nodes_max + i] += d.segc[b * S].w * esum / vol;  // n_e <eps>
        }
    }
    if (tid == 0) {
        ds.fe = fe;
        if (a.mode == kFinStep) {
            if (a.diag) {
                ds.avg_samples += 1.0;
                ds.eepf_samples += 1.0;
            }
            ds.step += 1;
        }
    }
}

hipError_t launch_finalize(const FinArgs& a, hipStream_t st)
{
    const unsigned g = a.only_b >= 0 ? 1u : (unsigned)a.d.B;
    hipLaunchKernelGGL(finalize_kernel, dim3(g), dim3(kFinThreads), 0, st, a);
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
    const uint4 r0 = philox10((uint32_t)j, 0xFFFFFFFFu, ((uint32_t)a.s << 24) | 0u, (uint32_t)a.b,
                              dc.key0, dc.key1);
    const uint4 r1 = philox10((uint32_t)j, 0xFFFFFFFFu, ((uint32_t)a.s << 24) | 1u, (uint32_t)a.b,
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
    unsigned long long* acc = d.acc + ((size_t)b * d.S + s) * d.nodes_max;
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
