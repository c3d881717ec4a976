// Stable compaction of the particle slots: the live particles of every
// segment that has holes move, in their order, to the front of the other
// copy, and the copies swap.  Run every few steps (the push leaves holes where
// particles were absorbed).
//
// Tiles of 1024 slots (256 threads, 4 consecutive slots each), numbered over
// the segments that have holes.  Four plain passes, no waiting between
// workgroups (the two tile passes run on persistent grids):
//   count:   live particles of every tile
//   scan:    per segment, exclusive scan of its tiles' counts (first slot of
//            every tile), checked against the segment's live count
//   scatter: every live particle written to its tile's first slot + its rank
//            in the tile (four rounds of 256 neighbouring slots)
//   finish:  copies swap, count = live
#include "pic_device.h"
#include "pic_internal.h"
#include "pic_kernels.h"

#include <algorithm>

namespace pic {

namespace {

constexpr int kCT = 256;              // threads per compaction tile
constexpr int kCP = 4;                // slots per thread
constexpr int kCTile = kCT * kCP;

__device__ __forceinline__ bool has_holes(const DevPtrs& d, int g)
{
    return !d.diss[g / d.S].retired && d.segs[g].count != d.segs[g].live;
}

// first tile of every segment with holes (16 segments per lane at most), in LDS
__device__ __forceinline__ void hole_prefix(const DevPtrs& d, int32_t* pref)
{
    const int NS = d.B * d.S, lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        const int per = (NS + 63) >> 6, g0 = lane * per;
        int32_t run = 0;
        for (int j = 0; j < per; ++j) {
            const int g = g0 + j;
            if (g < NS) {
                if (has_holes(d, g)) run += (int32_t)((d.segs[g].count + kCTile - 1) / kCTile);
                pref[g + 1] = run;
            }
        }
        int32_t incl = run;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int32_t o = __shfl_up(incl, dd, 64);
            if (lane >= dd) incl += o;
        }
        const int32_t excl = incl - run;
        if (lane == 0) pref[0] = 0;
        for (int j = 0; j < per; ++j) {
            const int g = g0 + j;
            if (g < NS) pref[g + 1] += excl;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int seg_of_tile(const int32_t* pref, int NS, int32_t t)
{
    int lo = 0, hi = NS;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pref[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// live flags of this thread's slots
__device__ __forceinline__ uint32_t live_mask(const int32_t* cell, int64_t base, int64_t n)
{
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < kCP; ++j)
        if (base + j < n && cell[base + j] >= 0) m |= 1u << j;
    return m;
}

// exclusive scan over the workgroup of v; total in *tot
__device__ __forceinline__ uint32_t block_excl(uint32_t v, uint32_t* s_w, uint32_t* tot)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan_u32(v);
    if (lane == 63) s_w[wid] = incl;
    __syncthreads();
    uint32_t wex = 0, t = 0;
#pragma unroll
    for (int w = 0; w < kCT / 64; ++w) {
        if (w < wid) wex += s_w[w];
        t += s_w[w];
    }
    *tot = t;
    return wex + incl - v;
}

__global__ __launch_bounds__(kCT) void compact_count_kernel(DevPtrs d)
{
    __shared__ int32_t pref[kMaxSeg + 1];
    __shared__ uint32_t s_w[kCT / 64];
    hole_prefix(d, pref);
    const int NS = d.B * d.S;
    for (int32_t t = (int32_t)blockIdx.x; t < pref[NS]; t += (int32_t)gridDim.x) {
        const int g = seg_of_tile(pref, NS, t);
        const SegConst& sc = d.segc[g];
        const SegState& st = d.segs[g];
        const int64_t base = (int64_t)(t - pref[g]) * kCTile + (int64_t)threadIdx.x * kCP;
        const uint32_t m = live_mask(sc.cell[st.parity], base, st.count);
        uint32_t tot;
        (void)block_excl((uint32_t)__popc(m), s_w, &tot);
        if (threadIdx.x == 0) d.ccnt[t] = tot;
        __syncthreads();                           // s_w is reused
    }
}

__global__ __launch_bounds__(1024) void compact_scan_kernel(DevPtrs d)
{
    __shared__ int32_t pref[kMaxSeg + 1];
    __shared__ uint32_t s_w[16];
    hole_prefix(d, pref);
    const int g = blockIdx.x;
    if (g >= d.B * d.S || !has_holes(d, g)) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int32_t t0 = pref[g], nt = pref[g + 1] - pref[g];
    uint32_t run = 0;
    for (int32_t r0 = 0; r0 < nt; r0 += 1024) {
        const int32_t i = r0 + (int32_t)threadIdx.x;
        const uint32_t v = i < nt ? d.ccnt[t0 + i] : 0u;
        const uint32_t incl = wave_incl_scan_u32(v);
        if (lane == 63) s_w[wid] = incl;
        __syncthreads();
        uint32_t wex = 0, tot = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wid) wex += s_w[w];
            tot += s_w[w];
        }
        if (i < nt) d.ccnt[t0 + i] = run + wex + incl - v;
        run += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && (int64_t)run != d.segs[g].live) atomicOr(&d.diss[g / d.S].flags, kFlagCell);
}

__global__ __launch_bounds__(kCT) void compact_scatter_kernel(DevPtrs d)
{
    __shared__ int32_t pref[kMaxSeg + 1];
    __shared__ uint32_t s_w[2][kCT / 64];
    hole_prefix(d, pref);
    const int NS = d.B * d.S;
    for (int32_t t = (int32_t)blockIdx.x; t < pref[NS]; t += (int32_t)gridDim.x) {
        const int g = seg_of_tile(pref, NS, t);
        const SegConst& sc = d.segc[g];
        const SegState& st = d.segs[g];
        const int in = st.parity, out = in ^ 1;
        const int64_t base = (int64_t)(t - pref[g]) * kCTile;
        // rounds of 256 consecutive slots: lanes read and write neighbours
        int64_t first = d.ccnt[t];
#pragma unroll
        for (int r = 0; r < kCP; ++r) {
            const int64_t i = base + r * kCT + threadIdx.x;
            const int32_t c = i < st.count ? sc.cell[in][i] : -1;
            const bool live = c >= 0;
            uint32_t tot;
            const int64_t dst = first + block_excl(live ? 1u : 0u, s_w[r & 1], &tot);
            if (live) {
                if (dst < st.live) {
                    sc.cell[out][dst] = c;
                    sc.off[out][dst] = sc.off[in][i];
                    sc.vx[out][dst] = sc.vx[in][i];
                    sc.vy[out][dst] = sc.vy[in][i];
                    sc.vz[out][dst] = sc.vz[in][i];
                    sc.id[out][dst] = sc.id[in][i];
                    if (sc.z[0]) sc.z[out][dst] = sc.z[in][i];
                } else {                           // cannot happen when the counts agree
                    atomicOr(&d.diss[g / d.S].flags, kFlagCell);
                }
            }
            first += tot;
        }
        __syncthreads();                           // s_w is reused
    }
}

__global__ __launch_bounds__(256) void compact_finish_kernel(DevPtrs d)
{
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= d.B * d.S || !has_holes(d, g)) return;
    SegState& st = d.segs[g];
    st.parity ^= 1;
    st.count = st.live;
}

// Population control of one species over every discharge (the swarm's
// replicas): where the species holds more than `above` live particles, each
// is kept with probability keep / live, by an integer test on a Philox draw
// keyed by its id and the step (call 7); a removed particle becomes a hole,
// counted in the segment's dead count (zero between steps), which
// thin_finish takes off the live count before the compaction.  The live
// count is only read here, so every workgroup uses the same probability.
__global__ __launch_bounds__(256) void thin_mark_kernel(DevPtrs d, int32_t s, int64_t above, int64_t keep)
{
    const int b = (int)blockIdx.y;
    const int g = b * d.S + s;
    if (d.diss[b].retired) return;
    const SegState& st = d.segs[g];
    const int64_t live = st.live;
    if (live <= above || live <= keep) return;
    const uint32_t t24 = (uint32_t)(((uint64_t)keep << 24) / (uint64_t)live);   // < 2^24
    const SegConst& sc = d.segc[g];
    const DisConst& dc = d.disc[b];
    const uint32_t step = (uint32_t)d.diss[b].step;
    int32_t* cell = sc.cell[st.parity];
    const uint32_t* id = sc.id[st.parity];
    const int64_t n = st.count;
    uint32_t removed = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (cell[i] < 0) continue;
        const uint4 r = philox10(id[i], step, ((uint32_t)s << 24) | 7u, 0u, dc.key0, dc.key1);
        if (!(odd24(r.x) < t24)) {
            cell[i] = -1;
            ++removed;
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) removed += (uint32_t)__shfl_xor((int)removed, m, 64);
    if ((threadIdx.x & 63) == 0 && removed)
        atomicAdd(reinterpret_cast<unsigned long long*>(&d.segs[g].dead), (unsigned long long)removed);
}

__global__ __launch_bounds__(256) void thin_finish_kernel(DevPtrs d, int32_t s)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= d.B) return;
    SegState& st = d.segs[b * d.S + s];
    if (st.dead > 0) {
        st.live -= st.dead;
        st.dead = 0;
    }
}

}  // namespace

hipError_t launch_thin(const DevPtrs& d, int32_t species, int64_t above, int64_t keep, int64_t max_count,
                       int64_t max_tiles, int n_cu, hipStream_t st)
{
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((max_count + 255) / 256, 1024));
    hipLaunchKernelGGL(thin_mark_kernel, dim3(gx, (unsigned)d.B), dim3(256), 0, st, d, species, above, keep);
    hipLaunchKernelGGL(thin_finish_kernel, dim3((unsigned)((d.B + 255) / 256)), dim3(256), 0, st, d, species);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_compact(d, max_tiles, n_cu, st);
}

hipError_t launch_compact(const DevPtrs& d, int64_t max_tiles, int n_cu, hipStream_t st)
{
    const int NS = d.B * d.S;
    // persistent grids: every workgroup builds the segment prefix once and
    // strides over the tiles
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(max_tiles, (int64_t)n_cu * 8));
    hipLaunchKernelGGL(compact_count_kernel, dim3(grid), dim3(kCT), 0, st, d);
    hipLaunchKernelGGL(compact_scan_kernel, dim3((unsigned)NS), dim3(1024), 0, st, d);
    hipLaunchKernelGGL(compact_scatter_kernel, dim3(grid), dim3(kCT), 0, st, d);
    hipLaunchKernelGGL(compact_finish_kernel, dim3((unsigned)((NS + 255) / 256)), dim3(256), 0, st, d);
    return hipGetLastError();
}

int64_t compact_tiles_for(int64_t padded_count) { return (padded_count + kCTile - 1) / kCTile; }

}  // namespace pic
