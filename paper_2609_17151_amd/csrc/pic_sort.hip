// Stable counting sort of the particles of one species by cell, in every
// discharge of a context (run every K steps so that the particles a workgroup
// streams through stay in a narrow window of cells: fewer deposit flushes,
// local gathers).
//
// Tiles of 1024 consecutive particles (256 threads, 4 rounds of 64 per wave).
//   count:   per tile, stable ranks of equal cells inside each wave from
//            ballots on the key bits, per-wave cell counters in LDS, and the
//            tile's count of every cell written to a tiles x cells table H
//   part:    sums of H over groups of tiles, per cell
//   base:    per discharge, exclusive scan of the groups per cell and of the
//            cell totals: the first slot of every (group, cell)
//   offsets: H rewritten in place as the first slot of every (tile, cell)
//   scatter: ranks recomputed, every particle written to
//            offset(tile, cell) + earlier waves' count + rank in its wave,
//            into the other copy; then the copies swap.
// Every step is a plain pass with no waiting between workgroups; particles
// with equal cells keep their order, so the result equals a stable sort.
// Holes (slots of absorbed particles, cell < 0) are dropped.
#include "pic_device.h"
#include "pic_internal.h"
#include "pic_kernels.h"

namespace pic {

namespace {

constexpr int kST = 256;             // threads per sort tile
constexpr int kSR = 4;               // rounds of 64 per wave
constexpr int kSTile = kST * kSR;    // particles per sort tile
constexpr int kGroups = 64;          // tile groups per segment for the column scan

struct SortArgs {
    DevPtrs d;
    int32_t s;
    uint32_t* H;          // [tiles][cells_max]
    uint32_t* part;       // [B][kGroups][cells_max]
    int32_t key_bits;
};

// tiles per segment (count / 1024), prefix over discharges, in LDS
__device__ __forceinline__ void seg_prefix(const DevPtrs& d, int s, int64_t* pref)
{
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        int64_t loc[4];
        int64_t run = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int bb = lane * 4 + j;
            const int64_t n = (bb < d.B && !d.diss[bb].retired) ? d.segs[bb * d.S + s].count : 0;
            run += (n + kSTile - 1) / kSTile;
            loc[j] = run;
        }
        int64_t incl = run;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int64_t o = __shfl_up(incl, dd, 64);
            if (lane >= dd) incl += o;
        }
        const int64_t excl = incl - run;
        if (lane == 0) pref[0] = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int bb = lane * 4 + j;
            if (bb < d.B) pref[bb + 1] = excl + loc[j];
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int seg_of(const int64_t* pref, int B, int64_t t)
{
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pref[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// lanes of this wave holding the same key (valid lanes only)
__device__ __forceinline__ uint64_t peers_of(uint32_t key, bool valid, int bits)
{
    uint64_t m = __ballot(valid);
    for (int k = 0; k < bits; ++k) {
        const bool bit = (key >> k) & 1u;
        const uint64_t bm = __ballot(bit);
        m &= bit ? bm : ~bm;
    }
    return valid ? m : 0ull;
}

// stable ranks of one wave's 4 x 64 particles; counters cnt[cell] of this
// wave (u16), keys in registers
__device__ __forceinline__ void wave_rank(const int32_t* cell, int64_t wbase, int64_t n, int bits,
                                          unsigned short* cnt, int32_t* key, uint32_t* rank)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < kSR; ++r) {
        const int64_t idx = wbase + r * 64 + lane;
        const int32_t kc = idx < n ? cell[idx] : -1;
        const bool valid = kc >= 0;                // holes (absorbed particles) are dropped
        const int32_t k = valid ? kc : 0;
        const uint64_t pe = peers_of((uint32_t)k, valid, bits);
        const uint32_t before = (uint32_t)__popcll(pe & lt);
        uint32_t cur = 0;
        if (valid) cur = cnt[k];
        // every lane read the count before the leader updates it
        __builtin_amdgcn_wave_barrier();
        if (valid && before == 0) cnt[k] = (unsigned short)(cur + __popcll(pe));
        __builtin_amdgcn_wave_barrier();
        key[r] = valid ? k : -1;
        rank[r] = cur + before;
    }
}

}  // namespace

__global__ __launch_bounds__(kST) void sort_count_kernel(SortArgs a)
{
    const DevPtrs& d = a.d;
    __shared__ int64_t pref[PIC_MAX_BATCH + 1];
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned short* cnt = reinterpret_cast<unsigned short*>(smem);   // [4][cells_max]
    seg_prefix(d, a.s, pref);
    const int64_t t = blockIdx.x;
    if (t >= pref[d.B]) return;
    const int b = seg_of(pref, d.B, t);
    const SegConst& sc = d.segc[b * d.S + a.s];
    const SegState& st = d.segs[b * d.S + a.s];
    const int nc = d.disc[b].n_cells, cm = d.cells_max;
    const int wid = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < 4 * cm; i += kST) cnt[i] = 0;
    __syncthreads();
    int32_t key[kSR];
    uint32_t rank[kSR];
    const int64_t base = (t - pref[b]) * kSTile;
    wave_rank(sc.cell[st.parity], base + wid * 64 * kSR, st.count, a.key_bits, cnt + wid * cm, key, rank);
    __syncthreads();
    uint32_t* row = a.H + (size_t)t * cm;
    for (int c = threadIdx.x; c < nc; c += kST)
        row[c] = (uint32_t)cnt[c] + cnt[cm + c] + cnt[2 * cm + c] + cnt[3 * cm + c];
}

__global__ __launch_bounds__(256) void sort_part_kernel(SortArgs a)
{
    const DevPtrs& d = a.d;
    __shared__ int64_t pref[PIC_MAX_BATCH + 1];
    seg_prefix(d, a.s, pref);
    const int b = blockIdx.z, g = blockIdx.y;
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int nc = d.disc[b].n_cells, cm = d.cells_max;
    if (c >= nc) return;
    const int64_t tf = pref[b], nt = pref[b + 1] - pref[b];
    const int64_t gs = (nt + kGroups - 1) / kGroups;
    const int64_t t0 = tf + (int64_t)g * gs, t1 = (t0 + gs < tf + nt) ? t0 + gs : tf + nt;
    uint32_t sum = 0;
    for (int64_t t = t0; t < t1; ++t) sum += a.H[(size_t)t * cm + c];
    a.part[((size_t)b * kGroups + g) * cm + c] = sum;
}

__global__ __launch_bounds__(1024) void sort_base_kernel(SortArgs a)
{
    const DevPtrs& d = a.d;
    const int b = blockIdx.x;
    const int nc = d.disc[b].n_cells, cm = d.cells_max;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __shared__ uint32_t s_tot[kMaxCells];
    __shared__ uint32_t s_w[16];
    uint32_t* P = a.part + (size_t)b * kGroups * cm;
    for (int c = threadIdx.x; c < nc; c += 1024) {
        uint32_t run = 0;
        for (int g = 0; g < kGroups; ++g) {
            const uint32_t v = P[(size_t)g * cm + c];
            P[(size_t)g * cm + c] = run;
            run += v;
        }
        s_tot[c] = run;
    }
    __syncthreads();
    // exclusive scan of the cell totals: contiguous runs of 4 per thread
    const int c0 = threadIdx.x * 4;
    uint32_t loc[4], run = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        loc[j] = run;
        if (c0 + j < nc) run += s_tot[c0 + j];
    }
    const uint32_t incl = wave_incl_scan_u32(run);
    if (lane == 63) s_w[wid] = incl;
    __syncthreads();
    uint32_t wo = 0;
    for (int w = 0; w < wid; ++w) wo += s_w[w];
    const uint32_t texcl = wo + incl - run;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (c0 + j < nc) s_tot[c0 + j] = texcl + loc[j];
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += 1024) {
        const uint32_t cb = s_tot[c];
        for (int g = 0; g < kGroups; ++g) P[(size_t)g * cm + c] += cb;
    }
}

__global__ __launch_bounds__(256) void sort_offsets_kernel(SortArgs a)
{
    const DevPtrs& d = a.d;
    __shared__ int64_t pref[PIC_MAX_BATCH + 1];
    seg_prefix(d, a.s, pref);
    const int b = blockIdx.z, g = blockIdx.y;
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int nc = d.disc[b].n_cells, cm = d.cells_max;
    if (c >= nc) return;
    const int64_t tf = pref[b], nt = pref[b + 1] - pref[b];
    const int64_t gs = (nt + kGroups - 1) / kGroups;
    const int64_t t0 = tf + (int64_t)g * gs, t1 = (t0 + gs < tf + nt) ? t0 + gs : tf + nt;
    uint32_t run = a.part[((size_t)b * kGroups + g) * cm + c];
    for (int64_t t = t0; t < t1; ++t) {
        const uint32_t v = a.H[(size_t)t * cm + c];
        a.H[(size_t)t * cm + c] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kST) void sort_scatter_kernel(SortArgs a)
{
    const DevPtrs& d = a.d;
    __shared__ int64_t pref[PIC_MAX_BATCH + 1];
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned short* cnt = reinterpret_cast<unsigned short*>(smem);   // [4][cells_max]
    seg_prefix(d, a.s, pref);
    const int64_t t = blockIdx.x;
    if (t >= pref[d.B]) return;
    const int b = seg_of(pref, d.B, t);
    const SegConst& sc = d.segc[b * d.S + a.s];
    const SegState& st = d.segs[b * d.S + a.s];
    const int nc = d.disc[b].n_cells, cm = d.cells_max;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < 4 * cm; i += kST) cnt[i] = 0;
    __syncthreads();
    int32_t key[kSR];
    uint32_t rank[kSR];
    const int in = st.parity, out = in ^ 1;
    const int64_t n = st.count;
    const int64_t base = (t - pref[b]) * kSTile;
    const int64_t wbase = base + wid * 64 * kSR;
    wave_rank(sc.cell[in], wbase, n, a.key_bits, cnt + wid * cm, key, rank);
    __syncthreads();
    // counts of earlier waves, per cell, in place (exclusive over waves)
    for (int c = threadIdx.x; c < nc; c += kST) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t v = cnt[w * cm + c];
            cnt[w * cm + c] = (unsigned short)run;
            run += v;
        }
    }
    __syncthreads();
    const uint32_t* off = a.H + (size_t)t * cm;
#pragma unroll
    for (int r = 0; r < kSR; ++r) {
        const int64_t idx = wbase + r * 64 + lane;
        if (key[r] < 0) continue;
        const int k = key[r];
        const int64_t dst = (int64_t)off[k] + cnt[wid * cm + k] + rank[r];
        if (dst < 0 || dst >= n) {                 // cannot happen when the counts agree
            atomicOr(&d.diss[b].flags, kFlagCell);
            continue;
        }
        sc.cell[out][dst] = k;
        sc.off[out][dst] = sc.off[in][idx];
        sc.vx[out][dst] = sc.vx[in][idx];
        sc.vy[out][dst] = sc.vy[in][idx];
        sc.vz[out][dst] = sc.vz[in][idx];
        sc.id[out][dst] = sc.id[in][idx];
        if (sc.z[0]) sc.z[out][dst] = sc.z[in][idx];
    }
    (void)nc;
}

__global__ void sort_swap_kernel(DevPtrs d, int s)
{
    const int b = threadIdx.x;
    if (b < d.B && !d.diss[b].retired) {
        SegState& st = d.segs[b * d.S + s];
        st.parity ^= 1;
        st.count = st.live;                        // the holes are gone
    }
}

hipError_t launch_sort(const DevPtrs& d, int s, int64_t max_tiles, void* scratch, size_t scratch_bytes,
                       hipStream_t st)
{
    int bits = 1;
    while ((1 << bits) < d.cells_max) ++bits;
    SortArgs a{};
    a.d = d;
    a.s = s;
    a.key_bits = bits;
    const size_t h_bytes = (size_t)max_tiles * d.cells_max * 4;
    const size_t p_bytes = (size_t)d.B * kGroups * d.cells_max * 4;
    if (h_bytes + p_bytes > scratch_bytes) return hipErrorInvalidValue;
    a.H = (uint32_t*)scratch;
    a.part = (uint32_t*)((char*)scratch + h_bytes);
    const size_t lds = (size_t)4 * d.cells_max * 2;
    const dim3 gc((unsigned)((d.cells_max + 255) / 256), kGroups, (unsigned)d.B);
    hipLaunchKernelGGL(sort_count_kernel, dim3((unsigned)max_tiles), dim3(kST), lds, st, a);
    hipLaunchKernelGGL(sort_part_kernel, gc, dim3(256), 0, st, a);
    hipLaunchKernelGGL(sort_base_kernel, dim3((unsigned)d.B), dim3(1024), 0, st, a);
    hipLaunchKernelGGL(sort_offsets_kernel, gc, dim3(256), 0, st, a);
    hipLaunchKernelGGL(sort_scatter_kernel, dim3((unsigned)max_tiles), dim3(kST), lds, st, a);
    hipLaunchKernelGGL(sort_swap_kernel, dim3(1), dim3(PIC_MAX_BATCH), 0, st, d, s);
    return hipGetLastError();
}

size_t sort_scratch_bytes(int64_t max_tiles, int B, int cells_max)
{
    return (size_t)max_tiles * cells_max * 4 + (size_t)B * kGroups * cells_max * 4;
}

int64_t sort_tiles_for(int64_t padded_count) { return (padded_count + kSTile - 1) / kSTile; }

}  // namespace pic
