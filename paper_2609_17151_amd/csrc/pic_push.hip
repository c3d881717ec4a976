// Fused particle kernel of one leapfrog step for every species of every
// discharge of a context, in one launch (paper Section 1: explicit leapfrog,
// Boris pusher, walls and secondary emission, null-collision Monte Carlo with
// tabulated cross sections; the charge of the particles deposited on the mesh).
//
// Work is cut into tiles of T = threads * PPT consecutive particle slots of
// one (discharge, species) segment; tiles are numbered over all segments,
// discharge-major, and every workgroup takes a fixed contiguous range of
// tiles, so one launch covers the whole step with no waiting between
// workgroups.  Each thread owns PPT consecutive slots and moves them with
// 16-byte vector loads and stores, in place.  A workgroup stages the
// (E[c], E[c+1]) pairs of a discharge in LDS once per run of tiles of that
// discharge, and zeroes and flushes its deposit histogram once per run of
// tiles of one segment.
//
// Absorbed particles leave holes (cell = -1) that later steps skip; a stable
// compaction every few steps removes them.  Holes do not change the order of
// the live particles, and births are appended after the last slot in the
// order of their parents, so the particle order after a compaction is the
// order that compacting every step would give.  Births are staged per tile in
// particle order (a block scan of the birth flags) and appended by the
// finalize in tile order, which also gives their ids.
//
// Per particle: gather E by linear weighting, Boris push in the imposed B,
// cell-relative move in FP32, periodic wrap or absorption (with secondary
// emission for ions), the null-collision test and, for candidates, the
// collision.  Deposition: LDS histogram in 64-bit fixed point flushed with
// integer atomics, so sums are exact and independent of the order of tiles and
// runs are bit-reproducible without global float atomics.
//
// Streaming instances (GENERAL = false) serve periodic runs without
// collisions, where nothing can be absorbed or born: no ids, holes or births.
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

template <int N, typename V, typename S>
__device__ __forceinline__ void vload(const S* __restrict__ p, S* out)
{
    if constexpr (N % 4 == 0) {
        typedef S NV __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int k = 0; k < N / 4; ++k) {
            const NV v = ((const PIC_GLOBAL NV*)(p))[k];
            out[4 * k + 0] = v.x;
            out[4 * k + 1] = v.y;
            out[4 * k + 2] = v.z;
            out[4 * k + 3] = v.w;
        }
    } else {                       // (2-wide vector loads measured 4 % slower here)
#pragma unroll
        for (int k = 0; k < N; ++k) out[k] = ((const PIC_GLOBAL S*)(p))[k];
    }
}

template <int N, typename V, typename S>
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
            ((PIC_GLOBAL NV*)(p))[k] = v;
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) ((PIC_GLOBAL S*)(p))[k] = in[k];
    }
}

// The births of a tile, staged in LDS as they happen; `pkey` is the slot of
// the parent in the tile, so the tile's canonical order is the order of keys.
// A staged birth is deposited at once: an ionization electron into the
// workgroup's histogram and its ion into species 1, a secondary electron into
// species 0.
// a collision candidate waiting for the tile's collision pass
struct CollQ {
    uint32_t key;                  // slot in the tile
    int32_t c;
    float f, ux, uy, uz;
    uint32_t pid;
};

struct BirthSink {
    Birth* b;
    uint32_t* key;
    unsigned int* n;
    int cap;
    uint32_t pkey;
    unsigned long long* hist;      // this segment's LDS histogram
    unsigned long long* acc_e;     // species 0 of the discharge
    unsigned long long* acc_i;     // species 1 of the discharge (null with electrons only)
};

__device__ __forceinline__ bool stage_birth(const BirthSink& k, const Birth& x)
{
    const unsigned int i = atomicAdd(k.n, 1u);
    if (i >= (unsigned)k.cap) return false;
    k.b[i] = x;
    k.key[i] = k.pkey;
    return true;
}

// A particle's step up to the collision test.  Returns whether it stays;
// secondary electrons go to `sink`; `cand` says whether it is a collision
// candidate (the collision itself is collide_particle, run for the
// candidates of a tile together).
template <bool GENERAL>
__device__ __forceinline__ bool advance(const DevPtrs& d, const SegConst& sc, const DisConst& dc,
                                        const PushArgs& a, int s, int b, uint32_t step,
                                        const float2* ep, unsigned int* s_cnt, unsigned long long* s_wen, int& c,
                                        float& f, float& ux, float& uy, float& uz, uint32_t pid, float& ke_sum,
                                        const BirthSink& sink, bool& cand)
{
    const int nc = dc.n_cells;
    const int periodic = dc.bc == PIC_BC_PERIODIC;
    if ((unsigned)c >= (unsigned)nc) {     // corrupt state: latch, park the particle
        atomicOr(&d.diss[b].flags, kFlagCell);
        c = 0;
        f = 0.0f;
    }
    // gather
    const float2 e2 = ep[c];
    const float ex = e2.x + f * (e2.y - e2.x) + sc.eext[0];
    const float ey = sc.eext[1], ez = sc.eext[2];
    // Boris: half kick, rotation, half kick
    const float qmh = sc.qmh;
    const float tx = sc.tv[0], ty = sc.tv[1], tz = sc.tv[2];
    const float sx = sc.sv[0], sy = sc.sv[1], sz = sc.sv[2];
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
    f += ux * sc.dtdx;
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
    if (periodic) {
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
        atomicAdd(&s_wen[wall], (unsigned long long)(sc.half_m_over_e * vnew2 * 1048576.0f));
        if (a.diag) {
            // impact energy: this species' histogram at this wall, and for
            // electrons the wall energy distribution
            const float eps = sc.half_m_over_e * vnew2;
            const int wb = (int)(eps * sc.wedf_inv_bin);
            if ((unsigned)wb < (unsigned)kEepfBins)
                atomicAdd(&d.wedf[(((size_t)b * d.S + s) * 2 + wall) * kEepfBins + wb], 1ull);
            const int bin = (int)(eps * a.eepf_inv_bin);
            if (s == 0 && (unsigned)bin < (unsigned)kEepfBins)
                atomicAdd(&d.eepf[((size_t)b * 2 + 1) * kEepfBins + bin], 1ull);
        }
        if (GENERAL && sc.emits) {
            const uint4 r4 = philox10(pid, step, ((uint32_t)s << 24) | 4u, 0u, dc.key0, dc.key1);
            if (odd24(r4.x) < sc.see_k) {
                const uint4 r5 = philox10(pid, step, ((uint32_t)s << 24) | 5u, 0u, dc.key0, dc.key1);
                const float vn = sc.vsee * sqrtf(-2.0f * logf(u01f(r4.y)));
                const float adv = u01f(r4.z) * vn * sc.dtdx_e;   // cells
                float g0, g1;
                box_muller_f(u01f(r5.x), u01f(r5.y), g0, g1);
                // placed u v_n dt into the gap from the wall it came from
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
                bool kept = false;
                if (bc_ >= 0 && bc_ < nc) {
                    Birth x;
                    x.cell = bc_;
                    x.off = fr;
                    x.vx = wall == 0 ? vn : -vn;
                    x.vy = sc.vsee * g0;
                    x.vz = sc.vsee * g1;
                    x.ivx = x.ivy = x.ivz = 0.0f;
                    kept = stage_birth(sink, x);
                    if (kept) {
                        global_deposit(sink.acc_e, bc_, fr, nc, periodic);
                        atomicAdd(&s_cnt[C_SEE0 + wall], 1u);
                    } else {
                        atomicOr(&d.diss[b].flags, kFlagCapacity);
                    }
                }
                if (!kept) atomicAdd(&s_cnt[C_DROP], 1u);
            }
        }
        return false;
    }
    if (!GENERAL || sc.nch == 0) return true;
    // null-collision Monte Carlo: integer candidate test on the first draw
    const uint4 r = philox10(pid, step, ((uint32_t)s << 24), 0u, dc.key0, dc.key1);
    cand = r.x < sc.t32;
    return true;
}

// The collision of a candidate: the energy (electrons: target at rest; ions:
// relative to a sampled neutral), the channel by the running sum of the
// tabulated frequencies against the second word of the first draw, then the
// kinematics of the channel; an ionization stages its pair in `sink`.
__device__ __forceinline__ void collide_particle(const DevPtrs& d, const SegConst& sc, const DisConst& dc, int s,
                                                 int b, uint32_t step, unsigned int* s_cnt, int c, float f,
                                                 float& ux, float& uy, float& uz, uint32_t pid,
                                                 const BirthSink& sink)
{
    const int nc = dc.n_cells;
    const int periodic = dc.bc == PIC_BC_PERIODIC;
    const uint4 r = philox10(pid, step, ((uint32_t)s << 24), 0u, dc.key0, dc.key1);
    atomicAdd(&s_cnt[C_CAND], 1u);
    float speed, eps;
    float nvx = 0.0f, nvy = 0.0f, nvz = 0.0f;
    if (!sc.ion_type) {
        const float v2 = ux * ux + uy * uy + uz * uz;
        speed = sqrtf(v2);
        eps = sc.half_m_over_e * v2;
    } else {
        const uint4 r3 = philox10(pid, step, ((uint32_t)s << 24) | 3u, 0u, dc.key0, dc.key1);
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
    // channel: the first k whose running sum of n_g sigma_k g / nu_max passes
    // u1, one pass over the table row (the full sum checks the bound)
    const float u1 = u01f(r.y);
    float cum = 0.0f;
    int ch = -1;
    {
        const float lx = (logf(fmaxf(eps, 1e-30f)) - sc.xs_ln0) * sc.xs_inv_dln;
        int i;
        float fr;
        if (!(lx > 0.0f)) {
            i = 0;
            fr = 0.0f;
        } else if (lx >= (float)(sc.xs_n - 1)) {
            i = sc.xs_n - 2;
            fr = 1.0f;
        } else {
            i = (int)lx;
            if (i > sc.xs_n - 2) i = sc.xs_n - 2;
            fr = lx - (float)i;
        }
        const float* r0 = sc.xs + (size_t)i * sc.nch;
        const float* r1 = r0 + sc.nch;
        for (int k = 0; k < sc.nch; ++k) {
            const float v = r0[k] + fr * (r1[k] - r0[k]);
            cum += ((eps < sc.th[k]) ? 0.0f : v) * speed;
            if (ch < 0 && u1 < cum) ch = k;
        }
    }
    if (cum > 1.0f) atomicAdd(&s_cnt[C_VIOL], 1u);
    if (ch < 0) {
        atomicAdd(&s_cnt[C_NULL], 1u);
        return;
    }
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
            const uint4 r1 = philox10(pid, step, ((uint32_t)s << 24) | 1u, 0u, dc.key0, dc.key1);
            const uint4 r2 = philox10(pid, step, ((uint32_t)s << 24) | 2u, 0u, dc.key0, dc.key1);
            const float avail = eps - sc.th[ch];
            const float eej = u01f(r1.x) * avail;
            enew = avail - eej;
            float edx, edy, edz;
            scatter_dir(dx_, dy_, dz_, 1.0f - 2.0f * u01f(r1.y), 6.283185307179586f * u01f(r1.z), edx, edy,
                        edz);
            const float vej = sqrtf(sc.two_e_over_m * eej);
            float g0, g1, g2, g3;
            box_muller_f(u01f(r2.x), u01f(r2.y), g0, g1);
            box_muller_f(u01f(r2.z), u01f(r2.w), g2, g3);
            Birth x;
            x.cell = c;
            x.off = f;
            x.vx = vej * edx;
            x.vy = vej * edy;
            x.vz = vej * edz;
            x.ivx = sc.vt_gas * g0;
            x.ivy = sc.vt_gas * g1;
            x.ivz = sc.vt_gas * g2;
            if (stage_birth(sink, x)) {
                lds_deposit(sink.hist, c, f, nc, periodic);
                if (sink.acc_i) global_deposit(sink.acc_i, c, f, nc, periodic);   // no ions in a swarm
            } else {
                atomicOr(&d.diss[b].flags, kFlagCapacity);
                atomicAdd(&s_cnt[C_DROP], 1u);
            }
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

// velocity moments of a particle at the nodes, fixed point (diagnostics)
__device__ __forceinline__ void moment_diag(const SegConst& sc, unsigned long long* fh, unsigned long long* mh, int c,
                                            float f, float ux, int nc, int periodic)
{
    const int c1 = (periodic && c + 1 == nc) ? 0 : c + 1;
    const float a = ux * sc.mscale1, b2 = ux * ux * sc.mscale2;
    const float w0 = 1.0f - f;
    atomicAdd(&fh[c], (unsigned long long)(long long)rintf(w0 * a));
    atomicAdd(&fh[c1], (unsigned long long)(long long)rintf(f * a));
    atomicAdd(&mh[c], (unsigned long long)(long long)rintf(w0 * b2));
    atomicAdd(&mh[c1], (unsigned long long)(long long)rintf(f * b2));
}

__device__ __forceinline__ void electron_diag(const SegConst& sc, const DisConst& dc, const PushArgs& a,
                                              unsigned long long* ehist, unsigned int* eepf, int c, float f,
                                              float ux, float uy, float uz, int nc, int periodic)
{
    const float eps = sc.half_m_over_e * (ux * ux + uy * uy + uz * uz);
    const float w1 = f * eps, w0 = eps - w1;
    const int c1 = (periodic && c + 1 == nc) ? 0 : c + 1;
    atomicAdd(&ehist[c], (unsigned long long)(w0 * 1048576.0f));
    atomicAdd(&ehist[c1], (unsigned long long)(w1 * 1048576.0f));
    if (c >= dc.bulk_lo && c < dc.bulk_hi) {
        const int bin = (int)(eps * a.eepf_inv_bin);
        if ((unsigned)bin < (unsigned)kEepfBins) atomicAdd(&eepf[bin], 1u);
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

}  // namespace

template <int PPT, int BS, bool GENERAL>
__global__ __launch_bounds__(BS) void push_kernel(PushArgs a)
{
    constexpr int kBS = BS;
    constexpr int T = kBS * PPT;
    constexpr int kBirthsPerTile = T / kBirthsDiv;
    const DevPtrs& d = a.d;
    const int S = d.S, NS = d.B * d.S;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t s_pref[kMaxSeg + 1];   // first tile of every segment (discharge-major)
    __shared__ unsigned int s_cnt[C_N];
    __shared__ unsigned long long s_wen[2];   // energy carried into each wall by the run (eV, 2^20)
    __shared__ float s_red[kBS / 64];
    // collisions and births of up to kPair tiles of one segment are handled
    // in one round (fuller waves on the collision path); the counters
    // alternate between rounds so that a round's reset never meets the next
    // round's appends.  The queue holds kQcap candidates (a few per cent of
    // the particles are candidates); one past it collides where it is found.
    constexpr int kPair = 8;
    constexpr int kQcap = T;
    constexpr int kSink = GENERAL ? kBirthsPerTile : 1;
    __shared__ Birth s_bb[kPair * kSink];     // births of the round's tiles, kSink per tile
    __shared__ uint32_t s_bkey[kPair * kSink];
    __shared__ unsigned int s_bn[2 * kPair];  // their counts: [round parity][tile of the round]
    __shared__ CollQ s_q[GENERAL ? kQcap : 1];       // collision candidates of the round
    __shared__ unsigned int s_nq[2];          // their count, by round parity

    // ---- tiles per segment, prefix over the segments (up to 16 per lane) -----
    if (wid == 0) {
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
    if (tid < C_N) s_cnt[tid] = 0;
    if (tid < 2) s_wen[tid] = 0ull;
    if (tid < 2 * kPair) s_bn[tid] = 0u;
    if (tid < 2) s_nq[tid] = 0u;
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
    int rp = 0, npend = 0;                    // round parity, tiles of the open round
    int32_t pend_t0 = 0, pend_tin0 = 0;       // the round's first tile (global, in its segment)
    float ke_run = 0.0f;
    // a fixed contiguous range of tiles per workgroup
    const int32_t chunk = (NT + (int32_t)gridDim.x - 1) / (int32_t)gridDim.x;
    const int32_t t_begin = (int32_t)blockIdx.x * chunk;
    const int32_t t_end = t_begin + chunk < NT ? t_begin + chunk : NT;

    // flush the run of tiles of segment cg: deposit, diagnostics, counters,
    // kinetic energy (ranges are fixed, so the grouping of the sums is too)
    auto flush = [&](int cg) {
        __syncthreads();
        const int cb = cg / S, cs = cg - cb * S;
        const DisConst& dcf = d.disc[cb];
        const int rep = blockIdx.x % kRep;
        unsigned long long* acc_s = d.acc + ((size_t)cg * kRep + rep) * d.nodes_max;
        for (int i = tid; i < dcf.n_nodes; i += kBS) {
            const unsigned long long v = hist[i];
            if (v) atomicAdd(&acc_s[i], v);
        }
        if (a.diag) {
            unsigned long long* ma = d.macc + (size_t)cg * 2 * d.nodes_max;
            for (int i = tid; i < dcf.n_nodes; i += kBS) {
                const unsigned long long v = fhist[i], w = mhist[i];
                if (v) atomicAdd(&ma[i], v);
                if (w) atomicAdd(&ma[d.nodes_max + i], w);
            }
        }
        if (a.diag && cs == 0) {
            unsigned long long* ea = d.eacc + (size_t)cb * d.nodes_max;
            for (int i = tid; i < dcf.n_nodes; i += kBS) {
                const unsigned long long v = ehist[i];
                if (v) atomicAdd(&ea[i], v);
            }
            unsigned long long* eg = d.eepf + (size_t)cb * 2 * kEepfBins;
            for (int i = tid; i < kEepfBins; i += kBS) {
                const unsigned int v = eepf[i];
                if (v) atomicAdd(&eg[i], (unsigned long long)v);
            }
        }
        unsigned long long* cnt = d.cnt + ((size_t)cg * kRep + rep) * C_N;
        if (tid < C_N) {
            const unsigned int v = s_cnt[tid];
            if (v) {
                atomicAdd(&cnt[tid], (unsigned long long)v);
                if (tid == C_ABS0 || tid == C_ABS1)
                    atomicAdd(reinterpret_cast<unsigned long long*>(&d.segs[cg].dead), (unsigned long long)v);
            }
            s_cnt[tid] = 0;
        }
        if (tid < 2) {
            const unsigned long long v = s_wen[tid];
            if (v) atomicAdd(&d.wen[(size_t)cg * 2 + tid], v);
            s_wen[tid] = 0ull;
        }
        if (a.diag) {
            const double kt = block_sum_f32<BS>(ke_run, s_red);
            if (tid == 0) d.ke_part[run_first] = 0.5 * d.segc[cg].mw_half * kt;
            ke_run = 0.0f;
        }
    };

    for (int32_t t = t_begin; t < t_end; ++t) {
        // segment of tile t: the last g with s_pref[g] <= t
        int lo = 0, hi = NS;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_pref[mid] <= t) lo = mid; else hi = mid;
        }
        const int sg = lo;
        const int b = sg / S, s = sg - b * S;
        const DisConst& dc = d.disc[b];
        if (sg != cur_g) {
            if (cur_g >= 0) flush(cur_g);
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
            __syncthreads();
            cur_g = sg;
            cur_b = b;
            run_first = t;
        }
        const int32_t tile_first = s_pref[sg];
        const int32_t ntiles = s_pref[sg + 1] - tile_first;
        const int32_t tin = t - tile_first;
        const SegConst& sc = d.segc[sg];
        SegState& st = d.segs[sg];
        const int64_t n = st.count;
        const int nc = dc.n_cells;
        const int periodic = dc.bc == PIC_BC_PERIODIC;
        const uint32_t step = (uint32_t)d.diss[b].step;
        const int io = st.parity;                 // updated in place
        const int64_t base = (int64_t)tin * T + (int64_t)tid * PPT;

        int32_t cell[PPT];
        float off[PPT], vx[PPT], vy[PPT], vz[PPT];
        uint32_t pid[PPT];
        vload<PPT, int4>(sc.cell[io] + base, cell);
        vload<PPT, float4>(sc.off[io] + base, off);
        vload<PPT, float4>(sc.vx[io] + base, vx);
        vload<PPT, float4>(sc.vy[io] + base, vy);
        vload<PPT, float4>(sc.vz[io] + base, vz);
        if (GENERAL) {
            vload<PPT, uint4>(sc.id[io] + base, pid);
        } else {
#pragma unroll
            for (int j = 0; j < PPT; ++j) pid[j] = 0u;
        }

        BirthSink sink;
        sink.b = s_bb + npend * kSink;
        sink.key = s_bkey + npend * kSink;
        sink.n = &s_bn[rp * kPair + npend];
        sink.cap = kBirthsPerTile;
        sink.hist = hist;
        sink.acc_e = d.acc + ((size_t)b * S + 0) * kRep * d.nodes_max;
        sink.acc_i = S > 1 ? d.acc + ((size_t)b * S + 1) * kRep * d.nodes_max : nullptr;
        float ke_tile = 0.0f;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (base + j >= n) continue;
            if (GENERAL && cell[j] < 0) continue;          // a hole: absorbed earlier
            sink.pkey = (uint32_t)(tid * PPT + j);
            bool cand = false;
            const bool keep = advance<GENERAL>(d, sc, dc, a, s, b, step, ep, s_cnt, s_wen, cell[j], off[j], vx[j],
                                               vy[j], vz[j], pid[j], ke_tile, sink, cand);
            if (GENERAL && keep && sc.renew_lz > 0.0f) {
                // axial transit: displacement along the third axis since
                // injection; past L_z, a fresh velocity from the species'
                // initial distribution (call 6) at the same x
                float* zp = sc.z[io] + base + j;
                float zz = *zp + vz[j] * sc.dt_f;
                if (fabsf(zz) >= sc.renew_lz) {
                    const uint4 r6 = philox10(pid[j], step, ((uint32_t)s << 24) | 6u, 0u, dc.key0, dc.key1);
                    float g0, g1, g2, g3;
                    box_muller_f(u01f(r6.x), u01f(r6.y), g0, g1);
                    box_muller_f(u01f(r6.z), u01f(r6.w), g2, g3);
                    vx[j] = sc.drift0[0] + sc.vth0 * g0;
                    vy[j] = sc.drift0[1] + sc.vth0 * g1;
                    vz[j] = sc.drift0[2] + sc.vth0 * g2;
                    zz = 0.0f;
                    atomicAdd(&s_cnt[C_REN], 1u);
                }
                *zp = zz;
            }
            if (keep) {
                lds_deposit(hist, cell[j], off[j], nc, periodic);
                const unsigned int q = (GENERAL && cand) ? atomicAdd(&s_nq[rp], 1u) : 0u;
                if (GENERAL && cand && q >= (unsigned)kQcap) {
                    // the round's queue is full: the collision happens here
                    collide_particle(d, sc, dc, s, b, step, s_cnt, cell[j], off[j], vx[j], vy[j], vz[j], pid[j],
                                     sink);
                    if (a.diag) {
                        moment_diag(sc, fhist, mhist, cell[j], off[j], vx[j], nc, periodic);
                        if (s == 0)
                            electron_diag(sc, dc, a, ehist, eepf, cell[j], off[j], vx[j], vy[j], vz[j], nc,
                                          periodic);
                    }
                } else if (GENERAL && cand) {
                    CollQ e;
                    e.key = sink.pkey | ((uint32_t)npend << 16);   // slot in the tile, tile of the round
                    e.c = cell[j];
                    e.f = off[j];
                    e.ux = vx[j];
                    e.uy = vy[j];
                    e.uz = vz[j];
                    e.pid = pid[j];
                    s_q[q] = e;
                } else if (a.diag) {
                    moment_diag(sc, fhist, mhist, cell[j], off[j], vx[j], nc, periodic);
                    if (s == 0)
                        electron_diag(sc, dc, a, ehist, eepf, cell[j], off[j], vx[j], vy[j], vz[j], nc, periodic);
                }
            } else {
                cell[j] = -1;                              // absorbed: leaves a hole
            }
        }
        ke_run += ke_tile;

        // in place; every particle keeps its slot
        if (base + PPT <= n) {
            vstore<PPT, int4>(sc.cell[io] + base, cell);
            vstore<PPT, float4>(sc.off[io] + base, off);
            vstore<PPT, float4>(sc.vx[io] + base, vx);
            vstore<PPT, float4>(sc.vy[io] + base, vy);
            vstore<PPT, float4>(sc.vz[io] + base, vz);
        } else {
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                if (base + j < n) {
                    sc.cell[io][base + j] = cell[j];
                    sc.off[io][base + j] = off[j];
                    sc.vx[io][base + j] = vx[j];
                    sc.vy[io][base + j] = vy[j];
                    sc.vz[io][base + j] = vz[j];
                }
            }
        }
        if (tid == 0 && tin == ntiles - 1) {
            st.tile_first = tile_first;
            st.ntiles = ntiles;
        }
        if (GENERAL) {
            if (npend == 0) {
                pend_t0 = t;
                pend_tin0 = tin;
            }
            ++npend;
            if (npend == kPair || tin == ntiles - 1 || t + 1 == t_end) {
                // the round's collisions together, with full lanes (a
                // candidate in the main loop would stall its whole wave on the
                // collision path); the new velocities overwrite the ones
                // stored above.  The round's tiles are consecutive.
                __threadfence_block();
                __syncthreads();
                const unsigned int nq = s_nq[rp] < (unsigned)kQcap ? s_nq[rp] : (unsigned)kQcap;
                for (unsigned int q = tid; q < nq; q += kBS) {
                    CollQ e = s_q[q];
                    const int pos = (int)(e.key >> 16);
                    BirthSink qs = sink;
                    qs.b = s_bb + pos * kSink;
                    qs.key = s_bkey + pos * kSink;
                    qs.n = &s_bn[rp * kPair + pos];
                    qs.pkey = e.key & 0xffffu;
                    collide_particle(d, sc, dc, s, b, step, s_cnt, e.c, e.f, e.ux, e.uy, e.uz, e.pid, qs);
                    const int64_t slot = (int64_t)(pend_tin0 + pos) * T + qs.pkey;
                    sc.vx[io][slot] = e.ux;
                    sc.vy[io][slot] = e.uy;
                    sc.vz[io][slot] = e.uz;
                    if (a.diag) {
                        moment_diag(sc, fhist, mhist, e.c, e.f, e.ux, nc, periodic);
                        if (s == 0) electron_diag(sc, dc, a, ehist, eepf, e.c, e.f, e.ux, e.uy, e.uz, nc, periodic);
                    }
                }
                __syncthreads();
                // each tile's births in the order of their parents' slots
                for (int pos = 0; pos < npend; ++pos) {
                    const unsigned int nst = s_bn[rp * kPair + pos];
                    const int nb = nst < (unsigned)kBirthsPerTile ? (int)nst : kBirthsPerTile;
                    const uint32_t* keys = s_bkey + pos * kSink;
                    const int32_t tt = pend_t0 + pos;
                    if (tid < nb) {
                        const uint32_t k = keys[tid];
                        int rank = 0;
                        for (int i = 0; i < nb; ++i) rank += keys[i] < k;
                        d.births[(size_t)tt * kBirthsPerTile + rank] = s_bb[pos * kSink + tid];
                    }
                    if (tid == 0) {
                        d.bcnt[tt] = nb;
                        if (nb) atomicAdd(reinterpret_cast<unsigned long long*>(&st.staged), (unsigned long long)nb);
                    }
                }
                __syncthreads();                  // the staged births are read
                if (tid == 0) {                   // free for the round after next
                    for (int pos = 0; pos < kPair; ++pos) s_bn[rp * kPair + pos] = 0u;
                    s_nq[rp] = 0u;
                }
                rp ^= 1;
                npend = 0;
            }
        }
    }
    if (cur_g >= 0) flush(cur_g);
}

#define PIC_KERNELS(X)   \
    X(1, 256, false)     \
    X(2, 256, false)     \
    X(4, 256, false)     \
    X(8, 256, false)     \
    X(4, 512, false)     \
    X(4, 1024, false)    \
    X(1, 256, true)      \
    X(2, 256, true)

#define PIC_INST(P, B, G) template __global__ void push_kernel<P, B, G>(PushArgs);
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

// nearest instantiated shape: general kernels run 256 threads and PPT <= 2;
// streaming kernels accept the shapes listed above
void push_shape(int& ppt, int& threads, bool general)
{
    if (general) {                // the collision path holds many registers: two per thread at most
        threads = 256;
        ppt = ppt >= 2 ? 2 : 1;
        return;
    }
    if (threads >= 1024) {
        threads = 1024;
        ppt = 4;
    } else if (threads >= 512) {
        threads = 512;
        ppt = 4;
    } else {
        threads = 256;
        ppt = ppt >= 8 ? 8 : (ppt >= 4 ? 4 : (ppt >= 2 ? 2 : 1));
    }
}

hipError_t launch_push(const PushArgs& a, int ppt, int threads, bool general, int64_t grid, hipStream_t st)
{
    const size_t lds = push_lds_bytes(a.nodes_max_dyn, a.cells_max_dyn, a.diag);
    const dim3 g((unsigned)grid);
#define PIC_LAUNCH(P, B, G)                                                              \
    if (ppt == P && threads == B && general == G) {                                      \
        hipLaunchKernelGGL((push_kernel<P, B, G>), g, dim3(B), lds, st, a);             \
        return hipGetLastError();                                                        \
    }
    PIC_KERNELS(PIC_LAUNCH)
#undef PIC_LAUNCH
    return hipErrorInvalidValue;
}

int push_occupancy(int ppt, int threads, bool general, size_t lds)
{
    int nb = 0;
#define PIC_OCC(P, B, G)                                                                            \
    if (ppt == P && threads == B && general == G) {                                                 \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(                                           \
                &nb, reinterpret_cast<const void*>(push_kernel<P, B, G>), B, lds) != hipSuccess)     \
            nb = 0;                                                                                 \
    }
    PIC_KERNELS(PIC_OCC)
#undef PIC_OCC
    return nb > 0 ? nb : 1;
}

}  // namespace pic
