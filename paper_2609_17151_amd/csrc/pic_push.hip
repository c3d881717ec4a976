// Fused particle kernel of one leapfrog step for one species over every
// discharge of a context (paper Section 1: explicit leapfrog, Boris pusher,
// walls and secondary emission, null-collision Monte Carlo with tabulated cross
// sections; the charge of the particles deposited on the mesh).
//
// One workgroup takes one tile of T = 256 * PPT consecutive particles of one
// (discharge, species) segment; each thread owns PPT consecutive particles and
// moves them with 16-byte vector loads.  Per particle: gather E (linear
// weighting from (E[c], E[c+1]) pairs staged in LDS), Boris push in the imposed
// B, cell-relative move in FP32, periodic wrap or absorption at the walls
// (with secondary emission for ions), the null-collision test and, for
// candidates, the collision.  Survivors are compacted in their original order
// and births appended in canonical order through a block prefix sum plus a
// decoupled look-back across tiles (tile ids are handed out in launch order by
// an atomic counter, so every tile waits only for tiles already running).
// Deposition: per-workgroup LDS histogram in 64-bit fixed point, flushed with
// integer atomics; integer sums make the result independent of the order of
// tiles, so runs are bit-reproducible without global float atomics.
#include "pic_device.h"
#include "pic_internal.h"
#include "pic_kernels.h"

namespace pic {

namespace {

constexpr int kBS = 256;
constexpr uint64_t kSurvMask = (1ull << 38) - 1;
constexpr int kBirthShift = 38;
constexpr uint64_t kBirthMask = (1ull << 24) - 1;
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint32_t kSpinLimit = 1u << 20;

// counters gathered per workgroup
enum { C_ABS0, C_ABS1, C_SEE0, C_SEE1, C_CAND, C_NULL, C_VIOL, C_DROP, C_COLL, C_N = C_COLL + kMaxChan };

struct Birth {
    int32_t cell;
    float off, vx, vy, vz;   // the electron (ionization or secondary)
    float ivx, ivy, ivz;     // the ion born with it (ionization only)
};

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

// sigma_k(eps) * n_g / nu_max from the uniform ln(eps) table, zero below threshold
__device__ __forceinline__ void xs_lookup(const SegConst& sc, float eps, float* out)
{
    float lx = (logf(fmaxf(eps, 1e-30f)) - sc.xs_ln0) * sc.xs_inv_dln;
    int i;
    float f;
    if (!(lx > 0.0f)) {
        i = 0;
        f = 0.0f;
    } else if (lx >= (float)(sc.xs_n - 1)) {
        i = sc.xs_n - 2;
        f = 1.0f;
    } else {
        i = (int)lx;
        if (i > sc.xs_n - 2) i = sc.xs_n - 2;
        f = lx - (float)i;
    }
    const float* r0 = sc.xs + (size_t)i * sc.nch;
    const float* r1 = r0 + sc.nch;
    for (int k = 0; k < sc.nch; ++k) {
        const float v = r0[k] + f * (r1[k] - r0[k]);
        out[k] = (eps < sc.th[k]) ? 0.0f : v;
    }
}

}  // namespace

template <int PPT, bool GENERAL>
__global__ __launch_bounds__(kBS) void push_kernel(PushArgs a)
{
    constexpr int T = kBS * PPT;
    const DevPtrs& d = a.d;
    const int s = a.species, S = d.S, B = d.B;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t s_pref[PIC_MAX_BATCH + 1];
    __shared__ int s_tile, s_b;
    __shared__ uint32_t s_wave[kBS / 64];
    __shared__ uint64_t s_excl_surv;
    __shared__ uint32_t s_excl_birth;
    __shared__ unsigned int s_cnt[C_N];
    __shared__ float s_ke[kBS / 64];

    const uint32_t par = (uint32_t)(d.diss[0].step & 1u);
    unsigned long long* status = d.status + ((size_t)s * 2 + par) * d.tiles_max;

    // ---- tile hand-out and segment lookup --------------------------------
    if (tid == 0) s_tile = (int)atomicAdd(&d.tile_ctr[s * 2 + par], 1u);
    if (wid == 0) {
        // prefix over discharges of tile counts (B <= 256: 4 per lane)
        int64_t loc[4];
        int64_t run = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = lane * 4 + j;
            const int64_t n = (b < B) ? d.segs[b * S + s].count : 0;
            run += (n + T - 1) / T;
            loc[j] = run;
        }
        int64_t incl = run;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int64_t o = __shfl_up(incl, dd, 64);
            if (lane >= dd) incl += o;
        }
        const int64_t excl = incl - run;
        if (lane == 0) s_pref[0] = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = lane * 4 + j;
            if (b < B) s_pref[b + 1] = excl + loc[j];
        }
    }
    if (tid < C_N) s_cnt[tid] = 0;
    __syncthreads();
    const int t = s_tile;
    if (tid == 0) {
        // the next step's chain words of this block id start cleared
        __hip_atomic_store(&d.status[((size_t)s * 2 + (par ^ 1u)) * d.tiles_max + blockIdx.x], 0ull,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (blockIdx.x == 0) d.tile_ctr[s * 2 + (par ^ 1u)] = 0u;
        int lo = 0, hi = B;  // find b with s_pref[b] <= t < s_pref[b+1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_pref[mid] <= t) lo = mid; else hi = mid;
        }
        s_b = lo;
    }
    __syncthreads();
    if ((int64_t)t >= s_pref[B]) return;
    const int b = s_b;
    const int64_t tile_first = s_pref[b];
    const int64_t ntiles = s_pref[b + 1] - tile_first;
    const int64_t tin = t - tile_first;       // tile index inside the segment
    const int sg = b * S + s;
    const SegConst& sc = d.segc[sg];
    SegState& st = d.segs[sg];
    const DisConst& dc = d.disc[b];
    const int64_t n = st.count;
    const int nc = dc.n_cells, nn = dc.n_nodes;
    const int periodic = dc.bc == PIC_BC_PERIODIC;
    const uint32_t step = (uint32_t)d.diss[b].step;
    const int in = st.parity;
    const int out = sc.compacts ? (in ^ 1) : in;

    // ---- LDS: E pairs and the deposit histogram ---------------------------
    unsigned long long* hist = reinterpret_cast<unsigned long long*>(smem);
    unsigned long long* ehist = hist + nn;                              // electron energy (diag)
    unsigned int* eepf = reinterpret_cast<unsigned int*>(ehist + (a.diag ? nn : 0));
    float2* ep = reinterpret_cast<float2*>(eepf + (a.diag ? kEepfBins : 0));
    const float2* epg = d.epair + (size_t)b * d.cells_max;
    for (int i = tid; i < nc; i += kBS) ep[i] = epg[i];
    for (int i = tid; i < nn; i += kBS) hist[i] = 0ull;
    if (a.diag) {
        for (int i = tid; i < nn; i += kBS) ehist[i] = 0ull;
        for (int i = tid; i < kEepfBins; i += kBS) eepf[i] = 0u;
    }
    __syncthreads();

    // ---- load PPT consecutive particles ----------------------------------
    const int64_t base = tin * T + (int64_t)tid * PPT;
    int32_t cell[PPT];
    float off[PPT], vx[PPT], vy[PPT], vz[PPT];
    uint32_t pid[PPT];
    const bool need_id = GENERAL || a.diag;
    {
        const int32_t* gc = sc.cell[in] + base;
        const float* go = sc.off[in] + base;
        const float* gx = sc.vx[in] + base;
        const float* gy = sc.vy[in] + base;
        const float* gz = sc.vz[in] + base;
        const uint32_t* gi = sc.id[in] + base;
        if constexpr (PPT == 4) {
            const int4 c4 = *reinterpret_cast<const int4*>(gc);
            const float4 o4 = *reinterpret_cast<const float4*>(go);
            const float4 x4 = *reinterpret_cast<const float4*>(gx);
            const float4 y4 = *reinterpret_cast<const float4*>(gy);
            const float4 z4 = *reinterpret_cast<const float4*>(gz);
            cell[0] = c4.x; cell[1] = c4.y; cell[2] = c4.z; cell[3] = c4.w;
            off[0] = o4.x; off[1] = o4.y; off[2] = o4.z; off[3] = o4.w;
            vx[0] = x4.x; vx[1] = x4.y; vx[2] = x4.z; vx[3] = x4.w;
            vy[0] = y4.x; vy[1] = y4.y; vy[2] = y4.z; vy[3] = y4.w;
            vz[0] = z4.x; vz[1] = z4.y; vz[2] = z4.z; vz[3] = z4.w;
            if (GENERAL) {
                const uint4 i4 = *reinterpret_cast<const uint4*>(gi);
                pid[0] = i4.x; pid[1] = i4.y; pid[2] = i4.z; pid[3] = i4.w;
            } else {
#pragma unroll
                for (int j = 0; j < PPT; ++j) pid[j] = 0;
            }
        } else if constexpr (PPT == 2) {
            const int2 c2 = *reinterpret_cast<const int2*>(gc);
            const float2 o2 = *reinterpret_cast<const float2*>(go);
            const float2 x2 = *reinterpret_cast<const float2*>(gx);
            const float2 y2 = *reinterpret_cast<const float2*>(gy);
            const float2 z2 = *reinterpret_cast<const float2*>(gz);
            cell[0] = c2.x; cell[1] = c2.y;
            off[0] = o2.x; off[1] = o2.y;
            vx[0] = x2.x; vx[1] = x2.y;
            vy[0] = y2.x; vy[1] = y2.y;
            vz[0] = z2.x; vz[1] = z2.y;
            if (GENERAL) {
                const uint2 i2 = *reinterpret_cast<const uint2*>(gi);
                pid[0] = i2.x; pid[1] = i2.y;
            } else {
                pid[0] = pid[1] = 0;
            }
        } else {
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                cell[j] = gc[j]; off[j] = go[j]; vx[j] = gx[j]; vy[j] = gy[j]; vz[j] = gz[j];
                pid[j] = GENERAL ? gi[j] : 0u;
            }
        }
        (void)need_id;
    }

    // ---- per-particle step -------------------------------------------------
    uint32_t alive = 0, born = 0;
    Birth bt[PPT];
    float ke_sum = 0.0f;
    const float qmh = sc.qmh;
    const float tx = sc.tv[0], ty = sc.tv[1], tz = sc.tv[2];
    const float sx = sc.sv[0], sy = sc.sv[1], sz = sc.sv[2];
    const float ex0 = sc.eext[0], ey = sc.eext[1], ez = sc.eext[2];
    const float dtdx = sc.dtdx;
    unsigned long long* acc_b = d.acc + ((size_t)b * S) * d.nodes_max;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        bt[j].cell = 0;
        bt[j].off = bt[j].vx = bt[j].vy = bt[j].vz = 0.0f;
        bt[j].ivx = bt[j].ivy = bt[j].ivz = 0.0f;
        const bool valid = base + j < n;
        if (!valid) continue;
        int c = cell[j];
        float f = off[j];
        if ((unsigned)c >= (unsigned)nc) {     // corrupt state: latch, park the particle
            atomicOr(&d.diss[b].flags, kFlagCell);
            c = 0;
            f = 0.0f;
        }
        // gather
        const float2 e2 = ep[c];
        const float ex = e2.x + f * (e2.y - e2.x) + ex0;
        // Boris
        float ux = vx[j], uy = vy[j], uz = vz[j];
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
        // move, cell-relative
        f += ux * dtdx;
        const float fl = floorf(f);
        c += (int)fl;
        f -= fl;
        if (f >= 1.0f) {
            f -= 1.0f;
            c += 1;
        }
        bool keep = true;
        if (!(f >= 0.0f && f < 1.0f) || !(fabsf(ux) < 3.0e38f)) {   // non-finite state
            atomicOr(&d.diss[b].flags, kFlagNumeric);
            f = 0.0f;
            c = 0;
            ux = uy = uz = 0.0f;
        }
        if (periodic) {
            if (c < 0) c += nc;
            else if (c >= nc) c -= nc;
            if ((unsigned)c >= (unsigned)nc) {                     // moved more than the domain
                atomicOr(&d.diss[b].flags, kFlagCell);
                c = 0;
                f = 0.0f;
            }
        } else if (c < 0 || c >= nc) {
            const int wall = c < 0 ? 0 : 1;
            keep = false;
            atomicAdd(&s_cnt[C_ABS0 + wall], 1u);
            if (a.diag && s == 0) {
                const float eps = sc.half_m_over_e * vnew2;
                const int bin = (int)(eps * a.eepf_inv_bin);
                if ((unsigned)bin < (unsigned)kEepfBins)
                    atomicAdd(&d.eepf[((size_t)b * 2 + 1) * kEepfBins + bin], 1ull);
            }
            if (GENERAL && sc.emits) {
                const uint4 r4 = philox10(pid[j], step, ((uint32_t)s << 24) | 4u, (uint32_t)b,
                                          dc.key0, dc.key1);
                if (odd24(r4.x) < sc.see_k) {
                    const uint4 r5 = philox10(pid[j], step, ((uint32_t)s << 24) | 5u, (uint32_t)b,
                                              dc.key0, dc.key1);
                    const float vn = sc.vsee * sqrtf(-2.0f * logf(u01f(r4.y)));
                    const float adv = u01f(r4.z) * vn * sc.dtdx_e;   // cells
                    float g0, g1;
                    box_muller_f(u01f(r5.x), u01f(r5.y), g0, g1);
                    // place the secondary u*v_n*dt into the gap from the wall
                    int bc_ = -1;
                    float fr = 0.0f;
                    if (adv < (float)nc) {
                        const float af = floorf(adv);
                        fr = adv - af;
                        if (wall == 0) {
                            bc_ = (int)af;
                        } else {
                            bc_ = nc - 1 - (int)af;
                            fr = 1.0f - fr;
                            if (fr >= 1.0f) {
                                fr -= 1.0f;
                                bc_ += 1;
                            }
                        }
                    }
                    if (bc_ >= 0 && bc_ < nc) {
                        bt[j].cell = bc_;
                        bt[j].off = fr;
                        bt[j].vx = wall == 0 ? vn : -vn;
                        bt[j].vy = sc.vsee * g0;
                        bt[j].vz = sc.vsee * g1;
                        born |= 1u << j;
                        atomicAdd(&s_cnt[C_SEE0 + wall], 1u);
                    } else {
                        atomicAdd(&s_cnt[C_DROP], 1u);
                    }
                }
            }
        }
        // null-collision Monte Carlo
        if (GENERAL && keep && sc.nch > 0) {
            const uint4 r = philox10(pid[j], step, ((uint32_t)s << 24), (uint32_t)b, dc.key0, dc.key1);
            if (r.x < sc.t32) {
                atomicAdd(&s_cnt[C_CAND], 1u);
                float nu[kMaxChan];
                float speed, eps;
                float nvx = 0.0f, nvy = 0.0f, nvz = 0.0f;
                if (!sc.ion_type) {
                    const float v2 = ux * ux + uy * uy + uz * uz;
                    speed = sqrtf(v2);
                    eps = sc.half_m_over_e * v2;
                } else {
                    const uint4 r3 = philox10(pid[j], step, ((uint32_t)s << 24) | 3u, (uint32_t)b,
                                              dc.key0, dc.key1);
                    float g0, g1, g2, g3;
                    box_muller_f(u01f(r3.x), u01f(r3.y), g0, g1);
                    box_muller_f(u01f(r3.z), u01f(r3.w), g2, g3);
                    nvx = sc.vt_gas * g0;
                    nvy = sc.vt_gas * g1;
                    nvz = sc.vt_gas * g2;
                    const float gx = ux - nvx, gy = uy - nvy, gz = uz - nvz;
                    const float g2s = gx * gx + gy * gy + gz * gz;
                    speed = sqrtf(g2s);
                    eps = sc.half_m_over_e * g2s;
                }
                xs_lookup(sc, eps, nu);
                float total = 0.0f;
                for (int k = 0; k < sc.nch; ++k) {
                    nu[k] *= speed;
                    total += nu[k];
                }
                if (total > 1.0f) atomicAdd(&s_cnt[C_VIOL], 1u);
                const float u1 = u01f(r.y);
                float cum = 0.0f;
                int ch = -1;
                for (int k = 0; k < sc.nch; ++k) {
                    cum += nu[k];
                    if (u1 < cum) {
                        ch = k;
                        break;
                    }
                }
                if (ch < 0) {
                    atomicAdd(&s_cnt[C_NULL], 1u);
                } else {
                    atomicAdd(&s_cnt[C_COLL + ch], 1u);
                    const float cos_chi = 1.0f - 2.0f * u01f(r.z);
                    const float phi = 6.283185307179586f * u01f(r.w);
                    const int kind = sc.kind[ch];
                    if (!sc.ion_type) {
                        const float inv = 1.0f / speed;
                        const float dx_ = ux * inv, dy_ = uy * inv, dz_ = uz * inv;
                        float ndx, ndy, ndz;
                        scatter_dir(dx_, dy_, dz_, cos_chi, phi, ndx, ndy, ndz);
                        float enew;
                        if (kind == PIC_XS_ELASTIC) {
                            enew = eps * (1.0f - sc.mr2 * (1.0f - cos_chi));
                        } else if (kind == PIC_XS_EXCITATION) {
                            enew = eps - sc.th[ch];
                        } else {
                            const uint4 r1 = philox10(pid[j], step, ((uint32_t)s << 24) | 1u,
                                                      (uint32_t)b, dc.key0, dc.key1);
                            const uint4 r2 = philox10(pid[j], step, ((uint32_t)s << 24) | 2u,
                                                      (uint32_t)b, dc.key0, dc.key1);
                            const float avail = eps - sc.th[ch];
                            const float eej = u01f(r1.x) * avail;
                            enew = avail - eej;
                            float edx, edy, edz;
                            scatter_dir(dx_, dy_, dz_, 1.0f - 2.0f * u01f(r1.y),
                                        6.283185307179586f * u01f(r1.z), edx, edy, edz);
                            const float vej = sqrtf(sc.two_e_over_m * eej);
                            float g0, g1, g2, g3;
                            box_muller_f(u01f(r2.x), u01f(r2.y), g0, g1);
                            box_muller_f(u01f(r2.z), u01f(r2.w), g2, g3);
                            bt[j].cell = c;
                            bt[j].off = f;
                            bt[j].vx = vej * edx;
                            bt[j].vy = vej * edy;
                            bt[j].vz = vej * edz;
                            bt[j].ivx = sc.vt_gas * g0;
                            bt[j].ivy = sc.vt_gas * g1;
                            bt[j].ivz = sc.vt_gas * g2;
                            born |= 1u << j;
                        }
                        enew = fmaxf(enew, 0.0f);
                        const float vs = sqrtf(sc.two_e_over_m * enew);
                        ux = vs * ndx;
                        uy = vs * ndy;
                        uz = vs * ndz;
                    } else if (kind == PIC_XS_ION_CX) {
                        ux = nvx;
                        uy = nvy;
                        uz = nvz;
                    } else {
                        const float cmx = sc.m_frac * ux + sc.M_frac * nvx;
                        const float cmy = sc.m_frac * uy + sc.M_frac * nvy;
                        const float cmz = sc.m_frac * uz + sc.M_frac * nvz;
                        const float st_ = sqrtf(fmaxf(0.0f, 1.0f - cos_chi * cos_chi));
                        float sp_, cp_;
                        sincosf(phi, &sp_, &cp_);
                        const float gg = sc.M_frac * speed;
                        ux = cmx + gg * cos_chi;
                        uy = cmy + gg * st_ * cp_;
                        uz = cmz + gg * st_ * sp_;
                    }
                }
            }
        }
        cell[j] = c;
        off[j] = f;
        vx[j] = ux;
        vy[j] = uy;
        vz[j] = uz;
        if (keep) {
            alive |= 1u << j;
            lds_deposit(hist, c, f, nc, periodic);
            if (a.diag && s == 0) {
                const float eps = sc.half_m_over_e * (ux * ux + uy * uy + uz * uz);
                const float w1 = f * eps, w0 = eps - w1;
                const int c1 = (periodic && c + 1 == nc) ? 0 : c + 1;
                atomicAdd(&ehist[c], (unsigned long long)(w0 * 1048576.0f));
                atomicAdd(&ehist[c1], (unsigned long long)(w1 * 1048576.0f));
                if (c >= a.bulk_lo && c < a.bulk_hi) {
                    const int bin = (int)(eps * a.eepf_inv_bin);
                    if ((unsigned)bin < (unsigned)kEepfBins) atomicAdd(&eepf[bin], 1u);
                }
            }
        }
    }

    // ---- births deposit (rare): electron-species births into species 0's
    // histogram / accumulator, ionization ions into species 1's accumulator
    if (GENERAL && born) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (!(born & (1u << j))) continue;
            if (s == 0) lds_deposit(hist, bt[j].cell, bt[j].off, nc, periodic);
            else global_deposit(acc_b, bt[j].cell, bt[j].off, nc, periodic);
            if (s == 0) global_deposit(acc_b + d.nodes_max, bt[j].cell, bt[j].off, nc, periodic);
        }
    }

    // ---- block scan of (survivors, births) --------------------------------
    uint32_t my_surv = __popc(alive), my_birth = __popc(born);
    uint32_t packed = my_surv | (my_birth << 16);
    uint32_t incl = wave_incl_scan_u32(packed);
    if (lane == 63) s_wave[wid] = incl;
    // kinetic-energy partial of the tile (fixed reduction order)
    float kw = wave_sum_f32(ke_sum);
    if (lane == 0) s_ke[wid] = kw;
    __syncthreads();
    uint32_t wexcl = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBS / 64; ++w) {
        if (w < wid) wexcl += s_wave[w];
        tot += s_wave[w];
    }
    const uint32_t texcl = wexcl + incl - packed;    // this thread's exclusive prefix
    const uint32_t agg_surv = tot & 0xFFFFu, agg_birth = tot >> 16;
    if (tid == 0) {
        double kt = 0.0;
        for (int w = 0; w < kBS / 64; ++w) kt += (double)s_ke[w];
        d.ke_part[(size_t)s * d.tiles_max + t] = 0.5 * sc.mw_half * kt;
    }

    // ---- look-back across the tiles of this segment -------------------------
    uint64_t excl_surv = 0;
    uint32_t excl_birth = 0;
    if (GENERAL) {
        if (wid == 0) {
            const uint64_t agg_word = (uint64_t)agg_surv | ((uint64_t)agg_birth << kBirthShift);
            if (tin == 0) {
                if (lane == 0)
                    __hip_atomic_store(&status[t], agg_word | kFlagInc, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            } else {
                if (lane == 0)
                    __hip_atomic_store(&status[t], agg_word | kFlagAgg, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                int64_t j0 = t - 1;
                uint64_t sum_s = 0, sum_b = 0;
                bool done = false;
                uint32_t spins = 0;
                while (!done) {
                    const int64_t jj = j0 - lane;
                    uint64_t w = kFlagInc;        // before the segment start: inclusive zero
                    if (jj >= tile_first)
                        w = __hip_atomic_load(&status[jj], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    while (__any((w >> 62) == 0)) {
                        __builtin_amdgcn_s_sleep(1);
                        if ((w >> 62) == 0 && jj >= tile_first)
                            w = __hip_atomic_load(&status[jj], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (++spins > kSpinLimit) {
                            if (lane == 0) atomicOr(&d.diss[b].flags, kFlagStall);
                            if ((w >> 62) == 0) w = kFlagInc;
                        }
                    }
                    const uint64_t incm = __ballot((w >> 62) == 2);
                    int last = 63;
                    if (incm) {
                        last = __ffsll((unsigned long long)incm) - 1;
                        done = true;
                    }
                    uint64_t vs_ = (lane <= last) ? (w & kSurvMask) : 0;
                    uint64_t vb_ = (lane <= last) ? ((w >> kBirthShift) & kBirthMask) : 0;
#pragma unroll
                    for (int dd = 32; dd >= 1; dd >>= 1) {
                        vs_ += __shfl_xor(vs_, dd, 64);
                        vb_ += __shfl_xor(vb_, dd, 64);
                    }
                    sum_s += vs_;
                    sum_b += vb_;
                    j0 -= 64;
                }
                excl_surv = sum_s;
                excl_birth = (uint32_t)sum_b;
                if (lane == 0) {
                    const uint64_t inc = ((excl_surv + agg_surv) & kSurvMask) |
                                         (((uint64_t)(excl_birth + agg_birth) & kBirthMask) << kBirthShift);
                    __hip_atomic_store(&status[t], inc | kFlagInc, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            if (lane == 0) {
                s_excl_surv = excl_surv;
                s_excl_birth = excl_birth;
            }
        }
        __syncthreads();
        excl_surv = s_excl_surv;
        excl_birth = s_excl_birth;
    }

    // ---- write survivors ----------------------------------------------------
    if (!sc.compacts) {
        // periodic: every particle stays at its index (in place)
        int32_t* gc = sc.cell[out] + base;
        float* go = sc.off[out] + base;
        float* gx = sc.vx[out] + base;
        float* gy = sc.vy[out] + base;
        float* gz = sc.vz[out] + base;
        if (PPT == 4 && base + 4 <= n) {
            *reinterpret_cast<int4*>(gc) = make_int4(cell[0], cell[1], cell[2], cell[3]);
            *reinterpret_cast<float4*>(go) = make_float4(off[0], off[1], off[2], off[3]);
            *reinterpret_cast<float4*>(gx) = make_float4(vx[0], vx[1], vx[2], vx[3]);
            *reinterpret_cast<float4*>(gy) = make_float4(vy[0], vy[1], vy[2], vy[3]);
            *reinterpret_cast<float4*>(gz) = make_float4(vz[0], vz[1], vz[2], vz[3]);
        } else {
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                if (base + j < n) {
                    gc[j] = cell[j]; go[j] = off[j]; gx[j] = vx[j]; gy[j] = vy[j]; gz[j] = vz[j];
                }
            }
        }
    } else {
        uint64_t pos = excl_surv + (texcl & 0xFFFFu);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (alive & (1u << j)) {
                sc.cell[out][pos] = cell[j];
                sc.off[out][pos] = off[j];
                sc.vx[out][pos] = vx[j];
                sc.vy[out][pos] = vy[j];
                sc.vz[out][pos] = vz[j];
                sc.id[out][pos] = pid[j];
                ++pos;
            }
        }
    }

    // ---- births into the staging buffers -------------------------------------
    if (GENERAL && born) {
        // species 0 births are ionization pairs (electron + ion); an ion
        // species' births are secondary electrons, placed after them.
        const int eseg = b * S + 0;
        const SegConst& se = d.segc[eseg];
        const int64_t base_e = (s == 0) ? 0 : d.segs[eseg].births;
        uint64_t k = (uint64_t)excl_birth + (texcl >> 16);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (!(born & (1u << j))) continue;
            const int64_t ke = base_e + (int64_t)k;
            if (ke < se.bcap) {
                se.bcell[ke] = bt[j].cell;
                se.boff[ke] = bt[j].off;
                se.bvx[ke] = bt[j].vx;
                se.bvy[ke] = bt[j].vy;
                se.bvz[ke] = bt[j].vz;
                se.bid[ke] = d.segs[eseg].next_id + (uint32_t)ke;
            } else {
                atomicOr(&d.diss[b].flags, kFlagCapacity);
            }
            if (s == 0) {
                const int iseg = b * S + 1;
                const SegConst& si = d.segc[iseg];
                if ((int64_t)k < si.bcap) {
                    si.bcell[k] = bt[j].cell;
                    si.boff[k] = bt[j].off;
                    si.bvx[k] = bt[j].ivx;
                    si.bvy[k] = bt[j].ivy;
                    si.bvz[k] = bt[j].ivz;
                    si.bid[k] = d.segs[iseg].next_id + (uint32_t)k;
                } else {
                    atomicOr(&d.diss[b].flags, kFlagCapacity);
                }
            }
            ++k;
        }
    }

    // ---- flush the deposit and counters --------------------------------------
    __syncthreads();
    unsigned long long* acc_s = acc_b + (size_t)s * d.nodes_max;
    for (int i = tid; i < nn; i += kBS) {
        const unsigned long long v = hist[i];
        if (v) atomicAdd(&acc_s[i], v);
    }
    if (a.diag) {
        unsigned long long* ea = d.eacc + (size_t)b * d.nodes_max;
        for (int i = tid; i < nn; i += kBS) {
            const unsigned long long v = ehist[i];
            if (v) atomicAdd(&ea[i], v);
        }
        unsigned long long* eg = d.eepf + (size_t)b * 2 * kEepfBins;
        for (int i = tid; i < kEepfBins; i += kBS) {
            const unsigned int v = eepf[i];
            if (v) atomicAdd(&eg[i], (unsigned long long)v);
        }
    }
    if (tid < C_N) {
        const unsigned int v = s_cnt[tid];
        if (v) {
            unsigned long long* dst = nullptr;
            switch (tid) {
                case C_ABS0: dst = &st.absorbed[0]; break;
                case C_ABS1: dst = &st.absorbed[1]; break;
                case C_SEE0: dst = &st.see[0]; break;
                case C_SEE1: dst = &st.see[1]; break;
                case C_CAND: dst = &st.cand; break;
                case C_NULL: dst = &st.nulls; break;
                case C_VIOL: dst = &st.viol; break;
                case C_DROP: dst = &st.dropped; break;
                default: dst = &st.coll[tid - C_COLL]; break;
            }
            atomicAdd(dst, (unsigned long long)v);
        }
    }
    // the last tile of the segment records the step's totals
    if (tid == 0 && tin == ntiles - 1) {
        st.tile_first = tile_first;
        st.ntiles = ntiles;
        st.surv = sc.compacts ? (int64_t)(excl_surv + agg_surv) : n;
        if (GENERAL) {
            const int64_t nb = (int64_t)excl_birth + agg_birth;
            if (s == 0) st.births = nb;      // ionization pairs
            else st.see_births = nb;         // secondaries (read by the finalize only)
        }
    }
}

template __global__ void push_kernel<1, false>(PushArgs);
template __global__ void push_kernel<2, false>(PushArgs);
template __global__ void push_kernel<4, false>(PushArgs);
template __global__ void push_kernel<1, true>(PushArgs);
template __global__ void push_kernel<2, true>(PushArgs);
template __global__ void push_kernel<4, true>(PushArgs);

size_t push_lds_bytes(int n_nodes, int n_cells, int diag)
{
    size_t b = (size_t)n_nodes * 8;
    if (diag) b += (size_t)n_nodes * 8 + kEepfBins * 4;
    b = (b + 15) & ~(size_t)15;
    b += (size_t)n_cells * 8;
    return b;
}

hipError_t launch_push(const PushArgs& a, int ppt, bool general, int64_t grid, hipStream_t st)
{
    const size_t lds = push_lds_bytes(a.nodes_max_dyn, a.cells_max_dyn, a.diag);
    dim3 g((unsigned)grid), blk(kBS);
#define PIC_LAUNCH(P, G) hipLaunchKernelGGL((push_kernel<P, G>), g, blk, lds, st, a)
    if (general) {
        if (ppt == 1) PIC_LAUNCH(1, true);
        else if (ppt == 2) PIC_LAUNCH(2, true);
        else PIC_LAUNCH(4, true);
    } else {
        if (ppt == 1) PIC_LAUNCH(1, false);
        else if (ppt == 2) PIC_LAUNCH(2, false);
        else PIC_LAUNCH(4, false);
    }
#undef PIC_LAUNCH
    return hipGetLastError();
}

}  // namespace pic
