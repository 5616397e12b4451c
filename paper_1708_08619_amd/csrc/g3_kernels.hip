// HIP kernels of libg3 for gfx950 (CDNA4, wave64).
//
// Pipeline per frame (Sec. 3.3; the paper's parallel g3 logic computes pair
// vectors first and then the triplets of each centre from them):
//   cell_count -> cell_scan -> cell_scatter      counting-sort cell build
//   nbr_build                                    minimum-image neighbour
//                                                vectors of every centre,
//                                                sorted by their pair bin
//   triplet (persistent) -> reduce               LDS-privatised r12 slabs,
//                                                flushed to uint64 bins
// Everything is integer: coordinates int32, squared distances uint32,
// LDS counters uint32, output uint64.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "g3_device.h"

namespace g3 {

namespace {

__device__ __forceinline__ size_t fr_off(const Sys& S, int f, size_t size)
{
    return S.per_frame ? (size_t)f * size : 0;
}

// floor(x nc / L) for 0 <= x < L <= 2^29, nc <= 2^10.  In double: x nc is
// exact, and a non-integer quotient lies at least 1/L > 2^-30 from the next
// integer while the rounded quotient is off by at most 2^-43, so the floor
// of the correctly rounded quotient is exact.
__device__ __forceinline__ int cell_of(int x, int nc, int L)
{
    return (int)((double)x * (double)nc / (double)L);
}

typedef short short2x __attribute__((ext_vector_type(2)));   // packed int16 pair

// Minimum image of one component (only used on axes with a single cell);
// |d| < L <= 2^29, so 2d fits int32.
__device__ __forceinline__ int min_image(int d, int L)
{
    const int d2 = 2 * d;
    return d2 > L ? d - L : (d2 < -L ? d + L : d);
}

// Exclusive scan over a 1024-thread block.  tmp needs 17 words.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t* total)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
    }
    if (lane == 63) tmp[w] = x;
    __syncthreads();
    if (w == 0) {
        uint32_t y = lane < nw ? tmp[lane] : 0u;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t t = __shfl_up(y, o, 64);
            if (lane >= o) y += t;
        }
        if (lane < nw) tmp[lane] = y;
    }
    __syncthreads();
    uint32_t pre = (w > 0 ? tmp[w - 1] : 0u) + x - v;
    *total = tmp[nw - 1];
    __syncthreads();
    return pre;
}

}  // namespace

// ------------------------------------------------------------------ utility
__global__ void k_zero_u32(uint32_t* p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Global-memory pointers.  Pointers read from a table (Sys) are generic, and
// generic accesses compile to flat instructions, which also count against the
// LDS wait counter: an LDS wait then waits for outstanding global loads and
// stores too.  Casting to the global address space gives global instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> gp(T* p)
{
    return (gptr<T>)p;
}
// (HIP's vector types assign through generic references only)
__device__ __forceinline__ void gstore(gptr<uint2> p, uint2 v)
{
    *(gptr<unsigned long long>)p = (unsigned long long)v.x | ((unsigned long long)v.y << 32);
}
__device__ __forceinline__ void gstore(gptr<int4> p, int4 v)
{
    typedef int int4v __attribute__((ext_vector_type(4)));
    *(gptr<int4v>)p = int4v{v.x, v.y, v.z, v.w};
}

// ------------------------------------------------------------------ cell build
// Validate coordinates, count atoms per cell and remember each atom's rank
// inside its cell (the atomic's return value).
__global__ void __launch_bounds__(256) k_cell_count(const Sys* __restrict__ sys,
                                                    const Job* __restrict__ jobs)
{
    const Job jb = jobs[blockIdx.y];
    const Sys& S = sys[jb.sys];
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= S.N) return;
    const int N = S.N, f = jb.frame;
    const gptr<const int32_t> fr = gp(S.frames + (size_t)f * 3 * N);
    const int x = fr[a], y = fr[N + a], z = fr[2 * N + a];
    if (x < 0 || x >= S.box[0] || y < 0 || y >= S.box[1] || z < 0 || z >= S.box[2]) {
        __hip_atomic_fetch_or(gp(&S.flags[f]), kFlagDomain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const int cell = (cell_of(z, S.nc[2], S.box[2]) * S.nc[1] + cell_of(y, S.nc[1], S.box[1])) *
                         S.nc[0] +
                     cell_of(x, S.nc[0], S.box[0]);
    const gptr<int32_t> cc = gp(S.cell_count + fr_off(S, f, S.ncell));
    // Lanes of a wave in the same cell share one atomic (frames stored in a
    // spatial order put many lanes in few cells); after 8 rounds the rest
    // take one atomic each.
    int rank = 0;
    bool todo = true;
    const int lane = threadIdx.x & 63;
    for (int round = 0; round < 8; ++round) {
        const uint64_t open = __ballot(todo);
        if (!open) break;
        const int leader = __builtin_ctzll(open);
        const int lc = __shfl(cell, leader, 64);
        const bool mine = todo && cell == lc;
        const uint64_t m = __ballot(mine);
        int base = 0;
        if (lane == leader)
            base = __hip_atomic_fetch_add(cc + lc, (int)__popcll(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        base = __shfl(base, leader, 64);
        if (mine) {
            rank = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            todo = false;
        }
    }
    if (todo) rank = __hip_atomic_fetch_add(cc + cell, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    gp(S.atom_cell)[fr_off(S, f, N) + a] = cell;
    gp(S.atom_rank)[fr_off(S, f, N) + a] = rank;
}

// Exclusive scan of the cell counts into cell_start[0..ncell].
__global__ void __launch_bounds__(1024) k_cell_scan(const Sys* __restrict__ sys,
                                                    const Job* __restrict__ jobs)
{
    __shared__ uint32_t tmp[17];
    const Job jb = jobs[blockIdx.x];
    const Sys& S = sys[jb.sys];
    const int f = jb.frame;
    const int32_t* cc = S.cell_count + fr_off(S, f, S.ncell);
    int32_t* cs = S.cell_start + fr_off(S, f, S.ncell + 1);
    uint32_t carry = 0;
    for (int base = 0; base < S.ncell; base += 1024) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < S.ncell ? (uint32_t)cc[i] : 0u;
        uint32_t tot;
        const uint32_t pre = block_excl_scan(v, tmp, &tot);
        if (i < S.ncell) cs[i] = (int32_t)(carry + pre);
        carry += tot;
    }
    if (threadIdx.x == 0) cs[S.ncell] = (int32_t)carry;
}

// Scatter coordinates into cell order (structure of arrays).
__global__ void __launch_bounds__(256) k_cell_scatter(const Sys* __restrict__ sys,
                                                      const Job* __restrict__ jobs)
{
    const Job jb = jobs[blockIdx.y];
    const Sys& S = sys[jb.sys];
    const int a = blockIdx.x * 256 + threadIdx.x;
    const int N = S.N, f = jb.frame;
    if (a >= N || (gp(S.flags)[f] & kFlagDomain)) return;
    const gptr<const int32_t> fr = gp(S.frames + (size_t)f * 3 * N);
    const int cell = gp(S.atom_cell)[fr_off(S, f, N) + a];
    const int pos = gp(S.cell_start)[fr_off(S, f, S.ncell + 1) + cell] + gp(S.atom_rank)[fr_off(S, f, N) + a];
    const gptr<int32_t> so = gp(S.sorted + fr_off(S, f, (size_t)3 * N));
    so[pos] = fr[a];
    so[N + pos] = fr[N + a];
    so[2 * N + pos] = fr[2 * N + a];
}

// ------------------------------------------------------------------ neighbours
// Workgroups loop over the cells of a frame.  The 27-cell stencil of the home
// cell is flattened into one list of candidate atoms whose coordinates carry
// the periodic shift of their stencil cell: with >= 3 cells on an axis and a
// cell side of at least C - 1 units that shift is the minimum image of every
// pair closer than rmax; an axis with a single cell gets an explicit minimum
// image.  The list is staged in LDS when it fits (else read from the
// cell-sorted arrays in global memory).  Each wave takes one centre:
//   pass 1 tests every candidate (|d|^2 < R2) and compacts the indices of
//   the accepted ones into a per-wave LDS list (ballot + mbcnt);
//   pass 2, on the accepted ones only, forms the entries and their pair
//   bins and r12 slabs: a short list is partitioned by slab in registers
//   (one ballot per slab), a longer one counts its slabs in LDS;
//   the list and its kListPad pad entries are reserved from the wave's chunk
//   of the frame's pool, the slab boundaries J_q are stored, and every
//   neighbour is written at J_{slab(b)} + its rank in the slab: the list
//   comes out partitioned by slab, which is all the triplet kernel needs.
// A centre with more neighbours than the buffer re-evaluates its candidates
// for the write.  Narrow staged candidates saturate their components to
// int16 and sum the squares with a clamped dot product; otherwise the
// components are tested against C before squaring (exact in uint32 for
// C <= 46340, products on the 24-bit multiplier).
namespace {

// The stencil of a cell: the home cell first, then the other cells.  In
// triangle-once mode an unordered pair belongs to one of its atoms: across
// two cells, to the atom from whose cell the other cell lies at a
// lexicographically positive offset (z first, then y, then x; stencil lanes
// run in that order, so these are the lanes after the home lane); within a
// cell, to the atom of lower cell-sorted index.  Every cell thus keeps 13
// neighbour cells, wherever the periodic grid wraps, and "atom j ranks above
// the centre" is simply t > tself.  Every component of an accepted side is
// at most C - 1, and cells are at least C - 1 wide, so seen from any atom of
// an accepted triangle the three cells sit at the same unwrapped offsets
// (each component -1, 0 or 1): the relation orders the three atoms totally
// and exactly one of them holds the other two in its list.
struct Stencil {
    int n;                 // stencil cells kept
    int start[27], pre[28];
    int shx[27], shy[27], shz[27];
};

// Orders the LDS traffic of one wave (lanes exchange data through LDS);
// global memory is not waited for.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
}


}  // namespace

constexpr int kBuildThreads = 512;
constexpr int kBuildWaves = kBuildWavesPerWG;
static_assert(kBuildThreads == 64 * kBuildWavesPerWG, "build workgroup shape");
// Neighbours buffered per wave before the write: 1 KB of entries per wave
// either way (a longer list re-evaluates its candidates for the write).
// Eight waves share a cell's staged stencil; at 35 KB of LDS and 71 VGPRs
// three workgroups (24 waves) share a CU (the kernel is latency-bound).
constexpr int kBufBytes = 1024;
template <bool WIDE>
constexpr int wave_buf() { return kBufBytes / (WIDE ? 16 : 8); }
constexpr int kWaveBufMax = kBufBytes / 8;
constexpr int kSplitSlabs = 8;    // slabs up to which a short list is partitioned in registers

// At most 64 VGPRs (8 waves per SIMD), so that four 8-wave workgroups share a
// CU: the build is latency-bound, and its few spills sit outside the pass-1 loop.
template <bool WIDE, bool ONE_STEP>
__global__ void __launch_bounds__(kBuildThreads, 8) k_nbr_build(const Sys* __restrict__ sys,
                                                             const Job* __restrict__ jobs, int list,
                                                             unsigned long long* cnt)
{
    using E = typename std::conditional<WIDE, int4, uint2>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* s_thr = reinterpret_cast<uint32_t*>(smem);                    // [kThrMax]
    uint8_t* s_tab = reinterpret_cast<uint8_t*>(s_thr + kThrMax);           // [8192]
    uint8_t* s_slab = s_tab + 8192;                                          // [256] bin -> slab
    constexpr int kWaveBuf = wave_buf<WIDE>();
    E* s_buf = reinterpret_cast<E*>(s_slab + 256);                           // [waves][kWaveBuf]
    uint32_t* s_scnt = reinterpret_cast<uint32_t*>(s_buf + kBuildWaves * kWaveBuf);  // [waves][64]
    uint32_t* s_g2 = s_scnt + kBuildWaves * 64;                              // [256] pair bins
    uint32_t* s_idx = s_g2 + 256;            // [waves][kWaveBufMax] candidate, then slab
    int32_t* s_x = reinterpret_cast<int32_t*>(s_idx + kBuildWaves * kWaveBufMax);  // [kStageCap]
    int32_t* s_y = s_x + kStageCap;
    int32_t* s_z = s_y + kStageCap;
    __shared__ Stencil st;

    const Job jb = jobs[blockIdx.y];
    const Sys& S = sys[jb.sys];
    const int f = jb.frame, N = S.N;
    if (gp(S.flags)[f] & kFlagDomain) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ncx = S.nc[0], ncy = S.nc[1], ncz = S.nc[2], ncell = S.ncell;
    const int Lx = S.box[0], Ly = S.box[1], Lz = S.box[2];
    const gptr<const int32_t> cs = gp(S.cell_start + fr_off(S, f, ncell + 1));
    const gptr<const int32_t> X = gp(S.sorted + fr_off(S, f, (size_t)3 * N));
    const gptr<const int32_t> Y = X + N;
    const gptr<const int32_t> Z = Y + N;
    const int cm1 = S.C - 1;
    const uint32_t span = 2u * (uint32_t)cm1;
    const uint32_t R2 = S.R2;
    const int sh = S.sh, nb = S.nbins, n_slabs = S.n_slabs, list_cap = S.list_cap;
    const int tbits = S.tab_bits;
    const int64_t pool_cap = S.pool_cap;
    uint32_t* scnt = s_scnt + wave * 64;
    E* buf = s_buf + wave * kWaveBuf;
    uint32_t* idx = s_idx + wave * kWaveBufMax;   // per buffered entry: candidate, then slab
    const gptr<uint32_t> flags = gp(S.flags + f);
    const gptr<uint32_t> cursor = gp(S.cursor + (size_t)f * kCursorStride);
    uint32_t chunk_base = 0, chunk_left = 0;   // this wave's slice of the pool
    const gptr<uint32_t> nbr_off = gp(S.nbr_off + fr_off(S, f, N));
    const gptr<uint32_t> nbr_cnt = gp(S.nbr_cnt + fr_off(S, f, N));
    const gptr<uint16_t> slab_j = gp(S.slab_j + fr_off(S, f, (size_t)N * (n_slabs + 1)));
    const size_t pbase = S.per_frame ? (size_t)f * (size_t)(pool_cap + kPoolPad) : 0;
    const gptr<E> pool = gp(reinterpret_cast<E*>(S.pool) + pbase);

    // bin tables and the bin -> slab map, once per workgroup
    const int nb3 = S.nb3;
    for (int x = tid; x <= nb3; x += kBuildThreads) s_thr[x] = gp(S.thr)[x];
    {
        const int n4 = (S.tab_len + 3) / 4;
        const gptr<const uint32_t> src = gp(reinterpret_cast<const uint32_t*>(S.tab));
        for (int x = tid; x < n4; x += kBuildThreads) reinterpret_cast<uint32_t*>(s_tab)[x] = src[x];
    }
    for (int b = tid; b < 256; b += kBuildThreads) {
        int q = 0;
        while (q + 1 < n_slabs && S.slab_lo[q + 1] <= b) ++q;
        s_slab[b] = (uint8_t)q;
        s_g2[b] = 0u;
    }
    // pair histogram (g2): accepted (centre, neighbour) pairs per bin, counted
    // in LDS and flushed with uint64 atomics before any counter could wrap
    uint64_t* const pair_hist = S.pair_hist;
    const bool tri_once = S.tri != nullptr;
    // triangle-once lists hold each unordered pair once (at its lower-ranked
    // atom): it stands for two ordered pairs
    const uint32_t pair_inc = tri_once ? 2u : 1u;
    uint64_t g2_pending = 0;   // upper bound on the counts held in s_g2
    auto flush_g2 = [&]() {
        for (int b = tid; b < nb; b += kBuildThreads) {
            const uint32_t v = s_g2[b];
            if (v) {
                __hip_atomic_fetch_add(gp(reinterpret_cast<unsigned long long*>(pair_hist + b)),
                                       (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_g2[b] = 0u;
            }
        }
    };
    const int rx = ncx >= 3 ? 1 : 0, ry = ncy >= 3 ? 1 : 0, rz = ncz >= 3 ? 1 : 0;
    const int nst = (2 * rx + 1) * (2 * ry + 1) * (2 * rz + 1);
    const int home = nst / 2;   // (0,0,0) sits in the middle of the odd stencil grid

    // The cells to build: all of the frame's, or (list) those the per-wave
    // build left in the frame's overflow list.
    const int n_items = list ? (int)gp(S.cursor)[(size_t)f * kCursorStride + kOvfWord] : ncell;
    const gptr<const int32_t> items = gp(S.ovf_cells + fr_off(S, f, ncell));
    // A cell's atom range and, in wave 0 (lane e: stencil offset e), its
    // stencil cells' index, start, end and periodic shift are loaded one cell
    // ahead, while the previous cell is processed.
    int p_c0 = 0, p_c1 = 0, p_c = 0x7fffffff, p_a = 0, p_e = 0, p_sx = 0, p_sy = 0, p_sz = 0;
    auto fetch_cell = [&](int k) {
        if (k >= n_items) return;
        const int cl = list ? items[k] : k;
        p_c0 = cs[cl];
        p_c1 = cs[cl + 1];
        if (wave == 0) {
            p_c = 0x7fffffff; p_a = 0; p_e = 0; p_sx = 0; p_sy = 0; p_sz = 0;
            if (lane < nst) {
                const int kx = cl % ncx, ky = (cl / ncx) % ncy, kz = cl / (ncx * ncy);
                const int ox = lane % (2 * rx + 1) - rx;
                const int oy = (lane / (2 * rx + 1)) % (2 * ry + 1) - ry;
                const int oz = lane / ((2 * rx + 1) * (2 * ry + 1)) - rz;
                int x = kx + ox, y = ky + oy, z = kz + oz;
                if (x < 0) { x += ncx; p_sx = -Lx; } else if (x >= ncx) { x -= ncx; p_sx = Lx; }
                if (y < 0) { y += ncy; p_sy = -Ly; } else if (y >= ncy) { y -= ncy; p_sy = Ly; }
                if (z < 0) { z += ncz; p_sz = -Lz; } else if (z >= ncz) { z -= ncz; p_sz = Lz; }
                p_c = (z * ncy + y) * ncx + x;
                p_a = cs[p_c];
                p_e = cs[p_c + 1];
            }
        }
    };
    fetch_cell(blockIdx.x);
    uint64_t n_tested = 0, n_found = 0;   // this wave's candidates and neighbours

    for (int k = blockIdx.x; k < n_items; k += gridDim.x) {
        const int c0 = p_c0, c1 = p_c1;
        const int a = p_a, e_end = p_e, shx = p_sx, shy = p_sy, shz = p_sz;
        fetch_cell(k + gridDim.x);
        if (c0 == c1) continue;   // uniform over the workgroup
        // stencil table: lane e of wave 0 takes stencil offset e; the home
        // cell goes to position 0, the kept others follow in lane order (the
        // cells are distinct), then a prefix sum of the counts in that order
        if (wave == 0) {
            const int cnt_e = lane < nst ? e_end - a : 0;
            // (triangle-once: the lexicographically positive offsets)
            const bool other = lane < nst && lane != home && (!tri_once || lane > home);
            const uint64_t om = __ballot(other);
            const int n_keep = 1 + (int)__popcll(om);
            int pos = -1;
            if (lane == home) pos = 0;
            if (other) pos = 1 + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(om >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)om, 0u));
            // counts in stencil order: lane p takes the count of the cell at p
            int v = 0;
            if (pos >= 0) {
                st.start[pos] = a;
                st.shx[pos] = shx; st.shy[pos] = shy; st.shz[pos] = shz;
                st.pre[pos] = cnt_e;                  // count, replaced by the prefix below
            }
            wave_sync();
            if (lane < n_keep) v = st.pre[lane];
            wave_sync();
            int incl = v;
#pragma unroll
            for (int d = 1; d < 32; d <<= 1) {
                const int y = __shfl_up(incl, d, 64);
                if (lane >= d) incl += y;
            }
            if (lane < n_keep) st.pre[lane] = incl - v;
            if (lane == n_keep - 1) { st.pre[n_keep] = incl; st.n = n_keep; }
        }
        __syncthreads();
        const int T = st.pre[st.n];
        const bool staged = T <= kStageCap;
        // stencil cell of candidate t: the last r < n with pre[r] <= t
        auto cell_of_t = [&](int t) {
            int r = 0;
            while (st.pre[r + 1] <= t) ++r;
            return r;
        };
        if (staged) {
            const int n_st = st.n;
            for (int t = tid; t < T; t += kBuildThreads) {
                // (the same, by binary search: pre is non-decreasing, n <= 27)
                int r = 0;
#pragma unroll
                for (int step = 16; step >= 1; step >>= 1)
                    if (r + step < n_st && st.pre[r + step] <= t) r += step;
                const int j = st.start[r] + (t - st.pre[r]);
                s_x[t] = X[j] + st.shx[r];
                s_y[t] = Y[j] + st.shy[r];
                s_z[t] = Z[j] + st.shz[r];
            }
        }
        __syncthreads();

        for (int ci = c0 + wave; ci < c1; ci += kBuildWaves) {
            // the centre is part of its own stencil (home cell: position 0,
            // no shift)
            const int tself = ci - st.start[0];
            // triangle-once mode keeps only the atoms ranked above the centre
            const int t_first = tri_once ? tself + 1 : 0;
            const int xi = staged ? s_x[tself] : X[ci];
            const int yi = staged ? s_y[tself] : Y[ci];
            const int zi = staged ? s_z[tself] : Z[ci];
            // Separation of candidate t from the centre; true if accepted.
            // Branch-free: an invalid candidate reads the centre's own
            // coordinates (staged) and is rejected.  Outside the narrow FAST
            // form every component is tested against C before the squares
            // are summed: with |d| <= C-1 narrow sums (C <= 32767) stay below
            // 2^32; wide ones (C <= 46340) may wrap only when dz^2 is added,
            // which the carry test catches.
            // MODE bit 0 (FAST): staged, and no axis needs an explicit minimum
            // image; bit 1: every candidate ranks above the centre
            // (triangle-once lists), so t != tself holds without a test.
            auto sep = [&](auto MODE, int t, int& dx, int& dy, int& dz, uint32_t& s) -> bool {
                constexpr bool FAST = (decltype(MODE)::value & 1) != 0;
                constexpr bool ABOVE = (decltype(MODE)::value & 2) != 0;
                const bool valid = t < T && (ABOVE || t != tself);
                int x, y, z;
                if (FAST || staged) {
                    const int tc = valid ? t : tself;
                    x = s_x[tc]; y = s_y[tc]; z = s_z[tc];
                } else {
                    if (!valid) return false;
                    const int r = cell_of_t(t);
                    const int j = st.start[r] + (t - st.pre[r]);
                    x = X[j] + st.shx[r]; y = Y[j] + st.shy[r]; z = Z[j] + st.shz[r];
                }
                dx = x - xi; dy = y - yi; dz = z - zi;
                if constexpr (!WIDE && FAST) {
                    // narrow (C <= 32767): components saturated to int16 and
                    // the squares summed with a clamped dot product; any
                    // saturated component or clamped sum is >= R2, and an
                    // accepted candidate's s is exact
                    const short2x pk = __builtin_amdgcn_cvt_pk_i16(dx, dy);
                    const int dzc = min(max(dz, -32768), 32767);
                    s = (uint32_t)__builtin_amdgcn_sdot2(pk, pk, __mul24(dzc, dzc), true);
                    return valid & (s < R2);
                }
                if constexpr (!FAST) {
                    if (ncx == 1) dx = min_image(dx, Lx);
                    if (ncy == 1) dy = min_image(dy, Ly);
                    if (ncz == 1) dz = min_image(dz, Lz);
                }
                const bool inr = max((uint32_t)(dx + cm1), max((uint32_t)(dy + cm1), (uint32_t)(dz + cm1))) <= span;
                const uint32_t s2 = (uint32_t)__mul24(dx, dx) + (uint32_t)__mul24(dy, dy);
                s = s2 + (uint32_t)__mul24(dz, dz);
                bool ok = valid & inr & (s < R2);
                if constexpr (WIDE) ok = ok & (s >= s2);
                return ok;
            };
            // pair bin of an accepted square distance s < R2
            auto bin_of = [&](uint32_t s) -> int {
                int b;
                if constexpr (ONE_STEP) {
                    b = s_tab[__builtin_amdgcn_ubfe(s, (uint32_t)sh, (uint32_t)tbits)];
                    b += (s >= s_thr[b + 1]) ? 1 : 0;
                } else {
                    b = s_tab[s >> sh];
                    while (s >= s_thr[b + 1]) ++b;
                }
                return b;
            };
            // entry after every list that no row accepts (see kListPad)
            auto pad_entry = [&]() -> E {
                if constexpr (WIDE) return make_int4(1 << 30, 1 << 30, 1 << 30, 0);
                else return make_uint2(0x80008000u, 0x00008000u);
            };
            auto pack = [&](int dx, int dy, int dz, int bn) -> E {
                if constexpr (WIDE) {
                    return make_int4(dx, dy, dz, bn);
                } else {
                    return make_uint2(((uint32_t)dx & 0xffffu) | ((uint32_t)dy << 16),
                                      ((uint32_t)dz & 0xffffu) | ((uint32_t)bn << 16));
                }
            };
            scnt[lane] = 0u;
            wave_sync();
            // Pass 1, the cheap one: test every candidate and compact the
            // indices of the accepted ones (a list longer than the buffer
            // overwrites its last index and is re-evaluated below).  Two
            // groups of 64 per iteration.
            uint32_t n = 0;
            auto push = [&](bool ok, int t) {
                const uint64_t mask = __ballot(ok);
                const uint32_t pos = n + __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                if (ok) idx[min(pos, (uint32_t)kWaveBuf - 1u)] = (uint32_t)t;
                n += (uint32_t)__popcll(mask);
            };
            // Pass 2, on the accepted candidates only: entry, pair bin, slab,
            // slab counts (and the pair histogram).  With at most 64 accepted
            // and at most kSplitSlabs slabs it is one sweep in registers: a
            // ballot per slab gives every entry its slab-partitioned position
            // and lane q the boundary J_q (the write follows the pool
            // reservation below); otherwise the slab counts go through LDS.
            E ent{};
            uint32_t epos = 0, jlane = 0;
            const bool split = n_slabs <= kSplitSlabs;
            auto pass12 = [&](auto MODE) {
                int t0 = t_first;
                for (; t0 + 64 < T; t0 += 128) {
                    int dx, dy, dz;
                    uint32_t sa, sb2;
                    const bool oa = sep(MODE, t0 + lane, dx, dy, dz, sa);
                    const bool ob = sep(MODE, t0 + 64 + lane, dx, dy, dz, sb2);
                    push(oa, t0 + lane);
                    push(ob, t0 + 64 + lane);
                }
                if (t0 < T) {   // at most 64 left: one group
                    int dx, dy, dz;
                    uint32_t sa;
                    push(sep(MODE, t0 + lane, dx, dy, dz, sa), t0 + lane);
                }
                wave_sync();
                if (split && n <= 64u) {
                    const bool act = (uint32_t)lane < n;
                    uint32_t q = 0xffu;
                    if (act) {
                        int dx, dy, dz;
                        uint32_t s;
                        sep(MODE, (int)idx[lane], dx, dy, dz, s);
                        const int b = bin_of(s);
                        q = s_slab[b];
                        if (pair_hist) atomicAdd(&s_g2[b], pair_inc);
                        ent = pack(dx, dy, dz, __mul24(b, nb3));
                    }
                    uint32_t J = 0;
                    for (int qq = 0; qq < n_slabs; ++qq) {
                        const bool mine = q == (uint32_t)qq;
                        const uint64_t mk = __ballot(mine);
                        if (lane == qq) jlane = J;
                        if (mine) epos = J + __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
                        J += (uint32_t)__popcll(mk);
                    }
                    if (lane == n_slabs) jlane = J;   // = n
                    return;
                }
                if (n > (uint32_t)kWaveBuf) return;
                for (uint32_t e = lane; e < n; e += 64) {
                    int dx, dy, dz;
                    uint32_t s;
                    sep(MODE, (int)idx[e], dx, dy, dz, s);
                    const int b = bin_of(s);
                    const uint32_t q = s_slab[b];
                    atomicAdd(&scnt[q], 1u);
                    if (pair_hist) atomicAdd(&s_g2[b], pair_inc);
                    buf[e] = pack(dx, dy, dz, __mul24(b, nb3));
                    idx[e] = q;
                }
            };
            const bool fast = staged && ncx > 1 && ncy > 1 && ncz > 1;
            if (fast && tri_once) pass12(std::integral_constant<int, 3>{});
            else if (fast) pass12(std::integral_constant<int, 1>{});
            else pass12(std::integral_constant<int, 0>{});
            wave_sync();
            n_tested += (uint64_t)(T - t_first - (tri_once ? 0 : 1));
            n_found += n;
            // a list longer than m_safe could take an item of the triplet
            // kernel past 2^32 candidate pairs: the frame is recomputed
            // with smaller items (its lists and pairs are still built here)
            if (n > (uint32_t)S.m_safe && lane == 0)
                __hip_atomic_fetch_or(flags, kFlagDense, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool in_regs = split && n <= 64u;
            const bool buffered = n <= (uint32_t)kWaveBuf;
            if (!in_regs && !buffered) {
                // a long list: count the slabs by re-evaluating every candidate
                for (int t0 = t_first; t0 < T; t0 += 64) {
                    int dx, dy, dz;
                    uint32_t s;
                    if (sep(std::false_type{}, t0 + lane, dx, dy, dz, s)) {
                        const int b = bin_of(s);
                        atomicAdd(&scnt[s_slab[b]], 1u);
                        if (pair_hist) atomicAdd(&s_g2[b], pair_inc);
                    }
                }
                wave_sync();
            }
            // a centre over the list capacity has its pairs counted, no list
            if (n > (uint32_t)list_cap) {
                if (lane == 0) {
                    __hip_atomic_fetch_or(flags, kFlagList, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    nbr_off[ci] = 0u;
                    nbr_cnt[ci] = 0u;
                }
                continue;
            }
            // bump-allocate from the wave's chunk (the list and its pad
            // entries); one global atomic per chunk
            const uint32_t nres = n ? n + (uint32_t)kListPad : 0u;
            if (nres > chunk_left) {
                const uint32_t want = nres > S.chunk ? nres : S.chunk;
                uint32_t got = 0;
                if (lane == 0) got = __hip_atomic_fetch_add(cursor, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                chunk_base = __shfl(got, 0, 64);
                chunk_left = want;
            }
            const uint32_t base = chunk_base;
            chunk_base += nres;
            chunk_left -= nres;
            if ((int64_t)base + nres > pool_cap) {
                if (lane == 0) __hip_atomic_fetch_or(flags, kFlagPool, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                continue;
            }
            if (in_regs) {
                if (lane <= n_slabs) slab_j[(size_t)ci * (n_slabs + 1) + lane] = (uint16_t)jlane;
                // entries and (one store) the pads that fit in the wave's lanes
                if (n && (uint32_t)lane < n + (uint32_t)kListPad)
                    gstore(pool + (base + ((uint32_t)lane < n ? epos : (uint32_t)lane)),
                           (uint32_t)lane < n ? ent : pad_entry());
                if (n + (uint32_t)kListPad > 64u && (uint32_t)lane < n + (uint32_t)kListPad - 64u)
                    gstore(pool + (base + 64u + lane), pad_entry());
                if (lane == 0) {
                    nbr_off[ci] = base;
                    nbr_cnt[ci] = n;
                }
                continue;
            }
            // slab boundaries J_q (exclusive scan of the slab counts)
            {
                const uint32_t v = lane < n_slabs ? scnt[lane] : 0u;
                uint32_t x = v;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t y = __shfl_up(x, d, 64);
                    if (lane >= d) x += y;
                }
                const uint32_t J = x - v;       // lane n_slabs gets the total n
                if (lane <= n_slabs) slab_j[(size_t)ci * (n_slabs + 1) + lane] = (uint16_t)J;
                wave_sync();
                if (lane < n_slabs) scnt[lane] = J;
                wave_sync();
            }
            // Pass 3: each entry at J_{slab} + its rank in the slab
            const gptr<E> P = pool + base;
            if (n && lane < kListPad) gstore(P + (n + lane), pad_entry());
            if (buffered) {
                for (uint32_t e = lane; e < n; e += 64) {
                    gstore(P + atomicAdd(&scnt[idx[e]], 1u), buf[e]);
                }
            } else {
                for (int t0 = t_first; t0 < T; t0 += 64) {
                    int dx, dy, dz;
                    uint32_t s;
                    if (sep(std::false_type{}, t0 + lane, dx, dy, dz, s)) {
                        const int b = bin_of(s);
                        gstore(P + atomicAdd(&scnt[s_slab[b]], 1u), pack(dx, dy, dz, __mul24(b, nb3)));
                    }
                }
            }
            if (lane == 0) {
                nbr_off[ci] = base;
                nbr_cnt[ci] = n;
            }
            wave_sync();
        }
        __syncthreads();   // the next cell restages s_x/s_y/s_z and st
        if (pair_hist) {       // uniform: cs and st are the same for every thread
            g2_pending += (uint64_t)(c1 - c0) * (uint64_t)T * pair_inc;
            if (g2_pending > 0x7fffffffull) {
                flush_g2();
                g2_pending = 0;
            }
        }
    }
    if (pair_hist && g2_pending) {
        __syncthreads();
        flush_g2();
    }
    if (cnt && lane == 0 && n_tested) {
        atomicAdd(cnt, (unsigned long long)n_tested);
        atomicAdd(cnt + 1, (unsigned long long)n_found);
    }
}

// ------------------------------------------------------------------ per-wave neighbours
// For narrow entries on a grid of >= 3 cells per axis whose stencil, taken
// relative to the home cell's midpoint, fits int16 (host: 1.5 cell widths
// plus a margin below 32767 units on every axis).  Every wave builds its own
// cells with its own stencil in LDS, so the main loop has no workgroup
// barrier:
//   the stencil (home cell first, then the kept neighbour cells, each atom
//   with its cell's periodic shift and the midpoint subtracted) is staged as
//   packed int16 coordinates (x | y << 16, z), followed by kStagePad
//   sentinel atoms at -32768 on every axis;
//   pass 1 tests 64 candidates per step: two saturating packed subtractions
//   and two clamped dot products give s = |d|^2, where a component beyond
//   int16 or a sum beyond int32 saturates to a value >= R2 (C <= 32767) and an
//   accepted s is exact; the sentinels are rejected by every centre, so no
//   bounds test is needed; the accepted staged indices are compacted
//   (ballot + mbcnt) into an index list as long as the stencil;
//   pass 2 forms the entries -- the packed difference IS the entry's first
//   word -- with their pair bins and r12 slabs, and writes the list
//   partitioned by slab exactly as the general build does.
// A cell whose stencil exceeds the wave's stage capacity, and every cell of a
// system without pk_ok, is appended to the frame's overflow list; the
// general build then runs on those cells only.  Workgroups of 4 waves on a
// 1-D grid: each job (one frame of one system) owns the workgroups from its
// wg0 to the next job's, in proportion to its cells.
namespace {

constexpr int kStagePad = 64;
constexpr uint32_t kWaveShared = 256;   // bin -> slab

struct WaveLds {   // byte offsets inside one wave's LDS region
    uint32_t stage, idx, scnt, g2, pre, start, offx, offy, offz, size;
};

// The stencil-cell table (pre, start, offx/y/z) is needed only while the
// stage is filled and the index list only after it, so the two share
// bytes; the pair-histogram counters exist only in launches that count
// pairs.  Seven 4-wave workgroups with a stage of 480 atoms and no pair
// counters then fit in one CU's LDS.
__host__ __device__ inline WaveLds wave_lds(int cap, bool g2)
{
    WaveLds w;
    uint32_t o = 0;
    w.stage = o; o += (uint32_t)(cap + kStagePad) * 8u;
    w.idx = o;
    w.pre = o;
    w.start = o + 32u * 4u;
    w.offx = o + 64u * 4u;
    w.offy = o + 96u * 4u;
    w.offz = o + 128u * 4u;
    const uint32_t ib = (uint32_t)cap * 2u > 160u * 4u ? (uint32_t)cap * 2u : 160u * 4u;
    o += (ib + 15u) & ~15u;
    w.scnt = o;  o += 64u * 4u;
    w.g2 = o;    o += g2 ? (uint32_t)kNbinsMax * 4u : 0u;
    w.size = o;
    return w;
}

typedef short short2p __attribute__((ext_vector_type(2)));

__device__ __forceinline__ short2p as_s2(uint32_t v) { return __builtin_bit_cast(short2p, v); }
__device__ __forceinline__ uint32_t as_u32(short2p v) { return __builtin_bit_cast(uint32_t, v); }

}  // namespace

template <int LOOKUP>
__global__ void __launch_bounds__(kWaveBuildWaves * 64, kWaveBuildMaxWgsPerCU) k_nbr_wave(const Sys* __restrict__ sys,
                                                                   const Job* __restrict__ jobs,
                                                                   int n_jobs, int cap, int with_g2,
                                                                   unsigned long long* cnt)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint8_t* s_slab = smem;                                                  // [256] bin -> slab
    const WaveLds WL = wave_lds(cap, with_g2 != 0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    unsigned char* wb = smem + kWaveShared + (size_t)wave * WL.size;
    uint2* stage = reinterpret_cast<uint2*>(wb + WL.stage);
    uint16_t* idx = reinterpret_cast<uint16_t*>(wb + WL.idx);
    uint32_t* scnt = reinterpret_cast<uint32_t*>(wb + WL.scnt);
    uint32_t* g2w = reinterpret_cast<uint32_t*>(wb + WL.g2);
    int32_t* st_pre = reinterpret_cast<int32_t*>(wb + WL.pre);
    int32_t* st_start = reinterpret_cast<int32_t*>(wb + WL.start);
    int32_t* st_ox = reinterpret_cast<int32_t*>(wb + WL.offx);
    int32_t* st_oy = reinterpret_cast<int32_t*>(wb + WL.offy);
    int32_t* st_oz = reinterpret_cast<int32_t*>(wb + WL.offz);

    // this workgroup's job: the last whose first workgroup is not after it
    int jl = 0, jh = n_jobs - 1;
    while (jl < jh) {
        const int mid = (jl + jh + 1) >> 1;
        if (jobs[mid].wg0 <= (int)blockIdx.x) jl = mid;
        else jh = mid - 1;
    }
    const Job jb = jobs[jl];
    const int wg_local = (int)blockIdx.x - jb.wg0;
    const int wg_count = (jl + 1 < n_jobs ? jobs[jl + 1].wg0 : (int)gridDim.x) - jb.wg0;
    const Sys& S = sys[jb.sys];
    const int f = jb.frame, N = S.N;
    if (gp(S.flags)[f] & kFlagDomain) return;   // uniform over the workgroup
    const int ncx = S.nc[0], ncy = S.nc[1], ncz = S.nc[2], ncell = S.ncell;
    const int Lx = S.box[0], Ly = S.box[1], Lz = S.box[2];
    const gptr<const int32_t> cs = gp(S.cell_start + fr_off(S, f, ncell + 1));
    const gptr<const int32_t> X = gp(S.sorted + fr_off(S, f, (size_t)3 * N));
    const gptr<const int32_t> Y = X + N;
    const gptr<const int32_t> Z = Y + N;
    const uint32_t R2 = S.R2;
    const int sh = S.sh, nb = S.nbins, n_slabs = S.n_slabs, nb3 = S.nb3;
    const int tbits = S.tab_bits;
    const int64_t pool_cap = S.pool_cap;
    const gptr<uint32_t> flags = gp(S.flags + f);
    const gptr<uint32_t> cursor = gp(S.cursor + (size_t)f * kCursorStride);
    const gptr<int32_t> ovf = gp(S.ovf_cells + fr_off(S, f, ncell));
    const gptr<uint32_t> nbr_off = gp(S.nbr_off + fr_off(S, f, N));
    const gptr<uint32_t> nbr_cnt = gp(S.nbr_cnt + fr_off(S, f, N));
    const gptr<uint16_t> slab_j = gp(S.slab_j + fr_off(S, f, (size_t)N * (n_slabs + 1)));
    const size_t pbase = S.per_frame ? (size_t)f * (size_t)(pool_cap + kPoolPad) : 0;
    const gptr<uint2> pool = gp(reinterpret_cast<uint2*>(S.pool) + pbase);
    // (a launch without pair counters has no system that counts pairs)
    uint64_t* const pair_hist = with_g2 ? S.pair_hist : nullptr;
    const bool tri_once = S.tri != nullptr;
    const uint32_t pair_inc = tri_once ? 2u : 1u;

    // the bin -> slab map, once per workgroup; the bin tables (a few KB) are
    // read through the vector cache, which keeps LDS for the stages (up to
    // seven 4-wave workgroups share a CU)
    const gptr<const uint32_t> g_thr = gp(S.thr);
    const gptr<const uint8_t> g_tab = gp(S.tab);
    const gptr<const uint32_t> g_step = gp(S.step);
    for (int b = tid; b < 256; b += kWaveBuildWaves * 64) {
        int q = 0;
        while (q + 1 < n_slabs && S.slab_lo[q + 1] <= b) ++q;
        s_slab[b] = (uint8_t)q;
    }
    if (with_g2)
        for (int b = lane; b < kNbinsMax; b += 64) g2w[b] = 0u;
    __syncthreads();   // the only workgroup barrier: waves work alone from here

    uint32_t g2_pending = 0;   // increments held in this wave's pair counters
    auto flush_g2 = [&]() {
        wave_sync();
        for (int b = lane; b < nb; b += 64) {
            const uint32_t v = g2w[b];
            if (v) {
                __hip_atomic_fetch_add(gp(reinterpret_cast<unsigned long long*>(pair_hist + b)),
                                       (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                g2w[b] = 0u;
            }
        }
        wave_sync();
        g2_pending = 0;
    };
    auto push_ovf = [&](int cell) {
        if (lane == 0) {
            const uint32_t k = __hip_atomic_fetch_add(cursor + kOvfWord, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            ovf[k] = cell;   // each cell is listed at most once: k < ncell
        }
    };
    auto bin_of = [&](uint32_t s) -> int {
        int b;
        if constexpr (LOOKUP == kLookupStepTable) {
            // one read: the cell's bin and the offset of its inner threshold
            const uint32_t ssh = (uint32_t)S.step_sh;
            b = (int)((g_step[__builtin_amdgcn_ubfe(s, ssh, (uint32_t)S.step_bits)] + s) >> ssh);
        } else if constexpr (LOOKUP == kLookupOneStep) {
            b = g_tab[__builtin_amdgcn_ubfe(s, (uint32_t)sh, (uint32_t)tbits)];
            b += (s >= g_thr[b + 1]) ? 1 : 0;
        } else {
            b = g_tab[s >> sh];
            while (s >= g_thr[b + 1]) ++b;
        }
        return b;
    };
    const uint2 pad_e = make_uint2(0x80008000u, 0x00008000u);   // pad entry after every list
    uint32_t chunk_base = 0, chunk_left = 0;   // this wave's slice of the frame's pool
    uint64_t n_tested = 0, n_found = 0;        // this wave's candidates and neighbours

    for (int cell = wg_local * kWaveBuildWaves + wave; cell < ncell; cell += wg_count * kWaveBuildWaves) {
        const int c0 = __builtin_amdgcn_readfirstlane(cs[cell]);
        const int c1 = __builtin_amdgcn_readfirstlane(cs[cell + 1]);
        if (c0 == c1) continue;
        if (!S.pk_ok) {
            push_ovf(cell);
            continue;
        }
        wave_sync();   // the previous cell's index list shares bytes with the cell table
        // stencil: lane e < 27 takes offset e; the home cell (e = 13) goes to
        // position 0, the kept others follow in lane order
        const int kx = cell % ncx, ky = (cell / ncx) % ncy, kz = cell / (ncx * ncy);
        // the home cell's midpoint (any point within a unit or two will do:
        // the host bound leaves a margin)
        const int refx = cell_mid(S.mid_q[0], kx);
        const int refy = cell_mid(S.mid_q[1], ky);
        const int refz = cell_mid(S.mid_q[2], kz);
        int ce = 0x7fffffff, ae = 0, ne = 0, ox = 0, oy = 0, oz = 0;
        if (lane < 27) {
            int x = kx + lane % 3 - 1, y = ky + (lane / 3) % 3 - 1, z = kz + lane / 9 - 1;
            int sx = 0, sy = 0, sz = 0;
            if (x < 0) { x += ncx; sx = -Lx; } else if (x >= ncx) { x -= ncx; sx = Lx; }
            if (y < 0) { y += ncy; sy = -Ly; } else if (y >= ncy) { y -= ncy; sy = Ly; }
            if (z < 0) { z += ncz; sz = -Lz; } else if (z >= ncz) { z -= ncz; sz = Lz; }
            ce = (z * ncy + y) * ncx + x;
            ae = cs[ce];
            ne = cs[ce + 1] - ae;
            ox = sx - refx; oy = sy - refy; oz = sz - refz;
        }
        // (triangle-once: the lexicographically positive offsets, lanes 14..26)
        const bool other = lane < 27 && lane != 13 && (!tri_once || lane > 13);
        const uint64_t om = __ballot(other);
        const int n_keep = 1 + (int)__popcll(om);
        int pos = -1;
        if (lane == 13) pos = 0;
        if (other) pos = 1 + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(om >> 32),
                                 __builtin_amdgcn_mbcnt_lo((uint32_t)om, 0u));
        if (pos >= 0) {
            st_start[pos] = ae;
            st_ox[pos] = ox; st_oy[pos] = oy; st_oz[pos] = oz;
            st_pre[pos] = ne;
        }
        wave_sync();
        const int v = lane < n_keep ? st_pre[lane] : 0;
        wave_sync();
        int incl = v;
#pragma unroll
        for (int d = 1; d < 32; d <<= 1) {
            const int y = __shfl_up(incl, d, 64);
            if (lane >= d) incl += y;
        }
        if (lane < n_keep) st_pre[lane] = incl - v;
        const int T = __builtin_amdgcn_readfirstlane(__shfl(incl, n_keep - 1, 64));
        if (T > cap) {          // stencil too large for this wave: general build
            push_ovf(cell);
            continue;
        }
        wave_sync();
        for (int t = lane; t < T + kStagePad; t += 64) {
            uint2 e = pad_e;      // sentinel: -32768 on every axis
            if (t < T) {
                int r = 0;
#pragma unroll
                for (int step = 16; step >= 1; step >>= 1)
                    if (r + step < n_keep && st_pre[r + step] <= t) r += step;
                const int j = st_start[r] + (t - st_pre[r]);
                const int x = X[j] + st_ox[r], y = Y[j] + st_oy[r], z = Z[j] + st_oz[r];
                e = make_uint2(((uint32_t)x & 0xffffu) | ((uint32_t)y << 16), (uint32_t)z & 0xffffu);
            }
            stage[t] = e;
        }
        wave_sync();

        const int Tu = T;
        for (int ci = c0; ci < c1; ++ci) {
            const int tself = ci - c0;      // the home cell is staged first, in cell order
            const uint2 cc = stage[tself];
            const short2p cxy = as_s2(cc.x), cz = as_s2(cc.y);
            // |d|^2 of staged atom t from the centre, saturated; the packed
            // differences are returned for the entry
            auto dist = [&](const uint2 e, short2p& dxy, short2p& dz) -> uint32_t {
                dxy = __builtin_elementwise_sub_sat(as_s2(e.x), cxy);
                dz = __builtin_elementwise_sub_sat(as_s2(e.y), cz);
                return (uint32_t)__builtin_amdgcn_sdot2(dz, dz, __builtin_amdgcn_sdot2(dxy, dxy, 0, true), true);
            };
            // Pass 1: test and compact the accepted staged indices (with
            // the triangle-once lists every candidate ranks above the centre;
            // otherwise the centre itself is excluded)
            uint32_t n = 0;
            auto pass1 = [&](auto TRI) {
                auto accept = [&](int t) -> bool {
                    short2p dxy, dz;
                    const bool ok = dist(stage[t], dxy, dz) < R2;
                    if constexpr (decltype(TRI)::value) return ok;
                    else return ok && t != tself;
                };
                auto push = [&](bool ok, int t) {
                    const uint64_t m = __builtin_amdgcn_ballot_w64(ok);
                    const uint32_t p = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)m, n));
                    if (ok) idx[p] = (uint16_t)t;
                    n += (uint32_t)__popcll(m);
                };
                int t0 = decltype(TRI)::value ? tself + 1 : 0;
                for (; t0 + 64 < Tu; t0 += 128) {
                    const bool oa = accept(t0 + lane);
                    const bool ob = accept(t0 + 64 + lane);
                    push(oa, t0 + lane);
                    push(ob, t0 + 64 + lane);
                }
                if (t0 < Tu) push(accept(t0 + lane), t0 + lane);
            };
            if (tri_once) pass1(std::true_type{});
            else pass1(std::false_type{});
            wave_sync();
            n_tested += (uint64_t)(tri_once ? Tu - tself - 1 : Tu - 1);
            n_found += n;
            // entry, pair bin and slab of accepted index e (slab via q)
            auto entry = [&](uint32_t e, int& b) -> uint2 {
                short2p dxy, dz;
                const uint32_t s = dist(stage[idx[e]], dxy, dz);
                b = bin_of(s);
                return make_uint2(as_u32(dxy), (as_u32(dz) & 0xffffu) | ((uint32_t)__mul24(b, nb3) << 16));
            };
            if (n > (uint32_t)S.m_safe && lane == 0)
                __hip_atomic_fetch_or(flags, kFlagDense, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (pair_hist) {
                if (g2_pending + n * pair_inc > 0x7fff0000u) flush_g2();
                g2_pending += n * pair_inc;
            }
            // bump-allocate the list and its pad entries from the wave's chunk
            const uint32_t nres = n ? n + (uint32_t)kListPad : 0u;
            if (nres > chunk_left) {
                const uint32_t want = nres > S.chunk ? nres : S.chunk;
                uint32_t got = 0;
                if (lane == 0) got = __hip_atomic_fetch_add(cursor, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                chunk_base = __shfl(got, 0, 64);
                chunk_left = want;
            }
            const uint32_t base = chunk_base;
            chunk_base += nres;
            chunk_left -= nres;
            const bool fits = (int64_t)base + nres <= pool_cap;
            if (!fits && lane == 0)
                __hip_atomic_fetch_or(flags, kFlagPool, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (n <= 64u && n_slabs <= kSplitSlabs) {
                // one sweep in registers: a ballot per slab gives every entry
                // its slab-partitioned position and lane q the boundary J_q
                const bool act = (uint32_t)lane < n;
                uint32_t q = 0xffu;
                uint2 ent = pad_e;
                if (act) {
                    int b;
                    ent = entry((uint32_t)lane, b);
                    q = s_slab[b];
                    if (pair_hist) atomicAdd(&g2w[b], pair_inc);
                }
                if (!fits) continue;
                uint32_t J = 0, epos = 0, jlane = 0;
                for (int qq = 0; qq < n_slabs; ++qq) {
                    const bool mine = q == (uint32_t)qq;
                    const uint64_t mk = __ballot(mine);
                    if (lane == qq) jlane = J;
                    if (mk) {   // (the innermost slabs are often empty)
                        if (mine) epos = __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mk, J));
                        J += (uint32_t)__popcll(mk);
                    }
                }
                if (lane == n_slabs) jlane = J;   // = n
                if (lane <= n_slabs) slab_j[(size_t)ci * (n_slabs + 1) + lane] = (uint16_t)jlane;
                if (n && (uint32_t)lane < n + (uint32_t)kListPad)
                    gstore(pool + (base + (act ? epos : (uint32_t)lane)), act ? ent : pad_e);
                if (n + (uint32_t)kListPad > 64u && (uint32_t)lane < n + (uint32_t)kListPad - 64u)
                    gstore(pool + (base + 64u + lane), pad_e);
                if (lane == 0) {
                    nbr_off[ci] = base;
                    nbr_cnt[ci] = n;
                }
                continue;
            }
            // longer list (or many slabs): count the slabs in LDS, scan, then
            // form the entries again and write each at its slab's cursor
            scnt[lane] = 0u;
            wave_sync();
            for (uint32_t e = lane; e < n; e += 64) {
                int b;
                (void)entry(e, b);
                atomicAdd(&scnt[s_slab[b]], 1u);
                if (pair_hist) atomicAdd(&g2w[b], pair_inc);
            }
            wave_sync();
            if (!fits) continue;
            {
                const uint32_t v = lane < n_slabs ? scnt[lane] : 0u;
                uint32_t x = v;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t y = __shfl_up(x, d, 64);
                    if (lane >= d) x += y;
                }
                const uint32_t J = x - v;       // lane n_slabs gets the total n
                if (lane <= n_slabs) slab_j[(size_t)ci * (n_slabs + 1) + lane] = (uint16_t)J;
                wave_sync();
                if (lane < n_slabs) scnt[lane] = J;
                wave_sync();
            }
            const gptr<uint2> P = pool + base;
            if (n && lane < kListPad) gstore(P + (n + lane), pad_e);
            for (uint32_t e = lane; e < n; e += 64) {
                int b;
                const uint2 ent = entry(e, b);
                gstore(P + atomicAdd(&scnt[s_slab[b]], 1u), ent);
            }
            if (lane == 0) {
                nbr_off[ci] = base;
                nbr_cnt[ci] = n;
            }
            wave_sync();
        }
    }
    if (pair_hist && g2_pending) flush_g2();
    if (cnt && lane == 0 && n_tested) {
        atomicAdd(cnt, (unsigned long long)n_tested);
        atomicAdd(cnt + 1, (unsigned long long)n_found);
    }
}

// ------------------------------------------------------------------ triplets
// Persistent workgroups pull items (system, r12 slab, frame, block of
// centres) from a device counter.  A workgroup keeps one slab of the
// histogram in LDS as uint32 counters while consecutive items share it, and
// flushes it to a partial slot (or, if slots run out, to the output with
// uint64 atomics) when the slab changes and at the end.
//
// Slab layout ("extended rows"): rows a in [lo0, lo1), columns b in
// [lo0, nbins), all c: index (a - lo0) * RL + (b - lo0) * nbins + c with
// RL = (nbins - lo0) * nbins.  An unordered pair is counted once, at
// (b_j, b_k) for the row j it was evaluated from; the reduce folds (a, b) and
// (b, a) into the half-layout bin (min, max, c).
//
// Per centre the neighbour list is partitioned by the r12 slab of its pair
// bins, slabs in increasing order (any order inside a slab).  The pairs whose
// smaller bin lies in the slab are those with at least one member among the
// slab rows, entries [J_q, J_q+1) (local 0..r-1 counted from J_q; m entries
// from J_q to the end of the list).  Row j takes k = j+1 .. m-1: the slab
// rows above it (each unordered pair of slab rows once, at its lower row)
// and every entry with bins >= lo1.  Rows j and r-1-j form one work unit of
// 2m - r - 1 candidates (the middle row of an odd r is a unit of its own), so
// the units of a centre are equally long and each is two contiguous runs.
// Per candidate: d_jk = d_ik - d_ij (no re-wrap), s = |d_jk|^2 exact,
// accepted iff s < R2, bin c from the table plus one threshold step.
namespace {

template <bool WIDE>
struct Ent;

template <>
struct Ent<false> {
    typedef uint2 T;
    typedef short short2v __attribute__((ext_vector_type(2)));
    // squared length of (k - j); saturating 16-bit differences and a clamped
    // dot product keep out-of-range candidates >= R2 (C <= 32767)
    static __device__ __forceinline__ uint32_t dist2(T vk, uint32_t jx, uint32_t jz, int)
    {
        const short2v dxy = __builtin_elementwise_sub_sat(__builtin_bit_cast(short2v, vk.x),
                                                          __builtin_bit_cast(short2v, jx));
        const short2v dzB = __builtin_elementwise_sub_sat(__builtin_bit_cast(short2v, vk.y),
                                                          __builtin_bit_cast(short2v, jz));
        const int dz = (int)dzB.x;
        return (uint32_t)__builtin_amdgcn_sdot2(dxy, dxy, dz * dz, true);
    }
    static __device__ __forceinline__ int col(T v) { return (int)(v.y >> 16); }
};

template <>
struct Ent<true> {
    typedef int4 T;
    // component pre-test against C, then s = dx^2 + dy^2 (+ dz^2): exact
    // in uint32 for C <= 46340; rejected candidates return 0xffffffff
    static __device__ __forceinline__ uint32_t dist2(T vk, int jx, int jy, int jz, int cm1)
    {
        const int dx = vk.x - jx, dy = vk.y - jy, dz = vk.z - jz;
        const uint32_t span = 2u * (uint32_t)cm1;
        if ((uint32_t)(dx + cm1) > span || (uint32_t)(dy + cm1) > span || (uint32_t)(dz + cm1) > span)
            return 0xffffffffu;
        const uint32_t s2 = (uint32_t)__mul24(dx, dx) + (uint32_t)__mul24(dy, dy);
        const uint32_t s = s2 + (uint32_t)__mul24(dz, dz);
        return s < s2 ? 0xffffffffu : s;   // s < s2 only if adding dz^2 wrapped
    }
    static __device__ __forceinline__ int col(T v) { return v.w; }
};

// Entries read straight from the neighbour pool with global (not flat)
// loads: a wave-uniform base plus a 32-bit byte offset per lane, so the
// loads take the scalar-base form and unrolled neighbours differ only in the
// immediate offset.
template <bool WIDE>
struct GEnt;

template <>
struct GEnt<false> {
    static constexpr uint32_t kSize = 8;
    typedef const __attribute__((address_space(1))) unsigned long long* P;
    typedef const __attribute__((address_space(1))) char* B;
    const char* base;   // uniform
    __device__ __forceinline__ uint2 load(uint32_t byte_off) const
    {
        const unsigned long long v = *(P)((B)base + byte_off);
        return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
    }
    // group of four consecutive entries from one 64-bit address
    __device__ __forceinline__ void load4(uint32_t byte_off, uint2 (&v)[4]) const
    {
        const P q = (P)((B)base + byte_off);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const unsigned long long x = q[u];
            v[u] = make_uint2((uint32_t)x, (uint32_t)(x >> 32));
        }
    }
};

template <>
struct GEnt<true> {
    static constexpr uint32_t kSize = 16;
    typedef int int4v __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) int4v* P;
    typedef const __attribute__((address_space(1))) char* B;
    const char* base;   // uniform
    __device__ __forceinline__ int4 load(uint32_t byte_off) const
    {
        const int4v v = *(P)((B)base + byte_off);
        return make_int4(v.x, v.y, v.z, v.w);
    }
    __device__ __forceinline__ void load4(uint32_t byte_off, int4 (&v)[4]) const
    {
        const P q = (P)((B)base + byte_off);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int4v x = q[u];
            v[u] = make_int4(x.x, x.y, x.z, x.w);
        }
    }
};

// LDS of the triplet kernel at fixed byte addresses.  The kernel declares no
// static LDS, so its dynamic LDS starts at address 0 (the host checks this
// before the first launch) and table bases fold into instruction offsets.
constexpr uint32_t kTlThr = 0;                        // uint32 thr[kThrMax]
constexpr uint32_t kTlTab = 4 * kThrMax;              // uint8 tab[kTabBytes]
constexpr uint32_t kTlTrash = kTlTab + kTabBytes;     // uint32 [64]: rejected candidates land here
constexpr uint32_t kTlMisc = kTlTrash + 256;          // uint32 scan[17], item, slot, chunk counter, flag
constexpr uint32_t kTlItem = kTlMisc + 4 * 17;
constexpr uint32_t kTlSlot = kTlItem + 4;
constexpr uint32_t kTlNext = kTlSlot + 4;
constexpr uint32_t kTlAny = kTlNext + 4;             // some centre of the item has rows
constexpr uint32_t kTlKeys = kTlMisc + 128;           // uint32 [256]: centres per row length
constexpr uint32_t kTlHist = kTlKeys + 1024;          // uint32 hist[hb_max], then per item:
                                                      // src[cb], m[cb], roff[cb+1], chunk[kChunkCap]
static_assert(kTlHist == kTripletLdsFixed, "triplet LDS map");
static_assert(kTripletThreads / kWave * 64 <= 1024, "each wave's 64 mark bytes fit the sort buckets");

// (LDS pointers are 32-bit on the device; the host pass sees 64-bit ones)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wint-to-pointer-cast"
typedef __attribute__((address_space(3))) uint32_t lds32_t;
typedef __attribute__((address_space(3))) uint16_t lds16_t;
typedef __attribute__((address_space(3))) uint8_t lds8_t;
__device__ __forceinline__ uint32_t ld32(uint32_t a) { return *(lds32_t*)a; }
__device__ __forceinline__ uint32_t ld16(uint32_t a) { return *(lds16_t*)a; }
__device__ __forceinline__ uint32_t ld8(uint32_t a) { return *(lds8_t*)a; }
__device__ __forceinline__ void st32(uint32_t a, uint32_t v) { *(lds32_t*)a = v; }
__device__ __forceinline__ void st16(uint32_t a, uint32_t v) { *(lds16_t*)a = (uint16_t)v; }
__device__ __forceinline__ void st8(uint32_t a, uint32_t v) { *(lds8_t*)a = (uint8_t)v; }
__device__ __forceinline__ void inc32(uint32_t a)
{
    __hip_atomic_fetch_add((lds32_t*)a, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t fetch_inc32(uint32_t a)
{
    return __hip_atomic_fetch_add((lds32_t*)a, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
#pragma clang diagnostic pop

// Exclusive scan over the 1024-thread block with its 17 scratch words at LDS
// address tmp.  Only LDS-address accessors are used: a generic pointer made
// from a fixed LDS address is not a valid LDS reference.
__device__ uint32_t block_excl_scan_at(uint32_t v, uint32_t tmp, uint32_t* total)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
    }
    if (lane == 63) st32(tmp + 4u * w, x);
    __syncthreads();
    if (w == 0) {
        uint32_t y = lane < nw ? ld32(tmp + 4u * lane) : 0u;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t t = __shfl_up(y, o, 64);
            if (lane >= o) y += t;
        }
        if (lane < nw) st32(tmp + 4u * lane, y);
    }
    __syncthreads();
    uint32_t pre = (w > 0 ? ld32(tmp + 4u * (w - 1)) : 0u) + x - v;
    *total = ld32(tmp + 4u * (nw - 1));
    __syncthreads();
    return pre;
}

}  // namespace

template <bool WIDE, int LOOKUP, bool PADDED>
__global__ void __launch_bounds__(kTripletThreads) k_triplet(TripletArgs A)
{
    using E = typename Ent<WIDE>::T;
    const uint32_t kSrc = kTlHist + 4u * (uint32_t)A.hb_max;
    const uint32_t kM = kSrc + 4u * (uint32_t)A.cb;
    const uint32_t kRoff = kM + 4u * (uint32_t)A.cb;
    const uint32_t kChunkT = kRoff + 4u * (uint32_t)(A.cb + 1);

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    int cur_seg = -1, cur_sys = -1;
    uint64_t pending = 0;    // upper bound on increments since the last flush
    uint64_t evaluated = 0;  // candidate pairs of the items this workgroup processed

    auto flush = [&](int seg) {
        const Seg& G = A.segs[seg];
        __syncthreads();
        if (tid == 0)
            st32(kTlSlot, __hip_atomic_fetch_add(gp(&A.ctl->slots_used), 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT));
        __syncthreads();
        const uint32_t slot = ld32(kTlSlot);
        if (slot < (uint32_t)A.max_slots) {
            const gptr<uint32_t> dst = gp(A.slots + (size_t)slot * A.hb_max);
            for (int x = tid; x < G.hb; x += kTripletThreads) dst[x] = ld32(kTlHist + 4u * x);
            if (tid == 0) A.slot_seg[slot] = seg;
        } else {
            // Fallback: add the non-zero bins directly; a wave skips 64 empty
            // bins with one ballot.
            const Sys& S = A.sys[G.sys];
            const int nb = S.nbins, nb3 = S.nb3, RL = G.rl;
            // triangle-once counts go to the half-layout triangle buffer
            const gptr<unsigned long long> out =
                gp(reinterpret_cast<unsigned long long*>(S.tri ? S.tri : S.hist));
            const int layout = S.tri ? 0 : S.layout;
            auto add = [](gptr<unsigned long long> p, unsigned long long v) {
                __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            };
            for (int x0 = wave * 64; x0 < G.hb; x0 += kTripletThreads) {
                const int x = x0 + lane;
                const uint32_t v = x < G.hb ? ld32(kTlHist + 4u * x) : 0u;
                if (__ballot(v != 0u) == 0ull) continue;
                if (v == 0u) continue;
                const int a = G.lo0 + x / RL, rem = x - (x / RL) * RL;
                const int b = G.lo0 + rem / nb3, c = rem - (rem / nb3) * nb3;
                const int lo = min(a, b), hi = max(a, b);
                if (layout == 0) {
                    const size_t h = ((size_t)lo * nb - (size_t)lo * (lo - 1) / 2 + (hi - lo)) * nb3 + c;
                    add(out + h, (unsigned long long)v);
                } else if (lo == hi) {
                    add(out + ((size_t)lo * nb + lo) * nb3 + c, 2ull * v);
                } else {
                    add(out + ((size_t)lo * nb + hi) * nb3 + c, (unsigned long long)v);
                    add(out + ((size_t)hi * nb + lo) * nb3 + c, (unsigned long long)v);
                }
            }
        }
        __syncthreads();
    };

    auto zero_hist = [&](int hb) {
        for (int x = tid; x < hb; x += kTripletThreads) st32(kTlHist + 4u * x, 0u);
    };

    // The counter hands out runs of consecutive items of one segment (a
    // segment's run length is `step`), so a workgroup keeps its slab over a
    // run.  Runs come in increasing order, so each workgroup finds the
    // segment of its next run by scanning forward from the last one.
    int seg = 0, item = 0, run_left = 0;
    for (;;) {
        if (tid == 0) {
            if (run_left == 0)
                st32(kTlItem, __hip_atomic_fetch_add(gp(&A.ctl->next_item), 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT));
            st32(kTlAny, 0u);
        }
        __syncthreads();
        if (run_left == 0) {
            const int fi = __builtin_amdgcn_readfirstlane((int)ld32(kTlItem));
            if (fi >= A.n_fetch) break;
            while (seg + 1 < A.n_segs && A.segs[seg + 1].fetch_begin <= fi) ++seg;
            const Seg& R = A.segs[seg];
            const int end = seg + 1 < A.n_segs ? A.segs[seg + 1].item_begin : A.total_items;
            item = R.item_begin + (fi - R.fetch_begin) * R.step;
            run_left = min(R.step, end - item);
        } else {
            ++item;
        }
        --run_left;
        __syncthreads();
        const Seg& G = A.segs[seg];
        const Sys& S = A.sys[G.sys];
        if (seg != cur_seg) {
            // (nothing added since the slab was zeroed: nothing to flush)
            if (cur_seg >= 0 && pending) flush(cur_seg);
            if (G.sys != cur_sys) {
                for (int x = tid; x <= S.nb3; x += kTripletThreads) st32(kTlThr + 4u * x, gp(S.thr)[x]);
                if constexpr (LOOKUP == kLookupStepTable)
                    for (int x = tid; x < S.step_len; x += kTripletThreads) st32(kTlTab + 4u * x, gp(S.step)[x]);
                else
                    for (int x = tid; x < S.tab_len; x += kTripletThreads) st8(kTlTab + x, gp(S.tab)[x]);
                cur_sys = G.sys;
            }
            zero_hist(G.hb);
            cur_seg = seg;
            pending = 0;
            __syncthreads();
        }
        const int local = item - G.item_begin;
        const int f = G.frame0 + local / G.n_blocks;
        const int blk = local - (local / G.n_blocks) * G.n_blocks;
        if (gp(S.flags)[f] != 0u) continue;
        const int N = S.N, q = G.slab, nb = S.nbins, lo0 = G.lo0;
        const int c_begin = blk * A.cb;
        const int nctr = min(A.cb, N - c_begin);
        const gptr<const uint32_t> off = gp(S.nbr_off + (S.per_frame ? (size_t)f * N : 0));
        const gptr<const uint32_t> cnt = gp(S.nbr_cnt + (S.per_frame ? (size_t)f * N : 0));
        const gptr<const uint16_t> J = gp(S.slab_j + (S.per_frame ? (size_t)f * N * (S.n_slabs + 1) : 0));
        const size_t pbase = S.per_frame ? (size_t)f * (size_t)(S.pool_cap + kPoolPad) : 0;
        const GEnt<WIDE> pool{reinterpret_cast<const char*>(S.pool) + pbase * sizeof(E)};
        constexpr uint32_t ES = GEnt<WIDE>::kSize;

        // per centre: its entries from J_q on (m) and its slab rows (r);
        // thread tid holds centres tid and tid + kTripletThreads of the item.
        // Centres with rows are put in order of decreasing row length (a
        // counting sort over 256 buckets), so that the 64 rows of a wave are
        // about equally long, and unit boundaries strictly increase.  The
        // item's candidate pairs stay below 2^32 (every uint32 counter exact):
        // the neighbour build flags frames with lists longer than m_safe.
        uint32_t m[kCentresPerThread], r[kCentresPerThread], src[kCentresPerThread],
            key[kCentresPerThread];
        uint32_t any = 0u;
#pragma unroll
        for (int h = 0; h < kCentresPerThread; ++h) {
            m[h] = r[h] = src[h] = key[h] = 0u;
            const int t = tid + h * kTripletThreads;
            if (t < nctr) {
                const int i = c_begin + t;
                const uint32_t o = off[i], n = cnt[i];
                const uint32_t j0 = J[(size_t)i * (S.n_slabs + 1) + q];
                const uint32_t j1 = J[(size_t)i * (S.n_slabs + 1) + q + 1];
                r[h] = j1 - j0;
                m[h] = r[h] ? n - j0 : 0u;
                src[h] = o + j0;
                key[h] = 255u - min(r[h] / 2u + (m[h] - r[h]), 255u);   // the centre's longest row
                any |= r[h];
            }
        }
        if (any) st32(kTlAny, 1u);
        if (tid < 256) st32(kTlKeys + 4u * tid, 0u);
        if (tid == 0) st32(kTlNext, 0u);
        __syncthreads();
        // a block with no rows in this slab (common for slabs at short
        // distances) skips the sort and the scans
        if (ld32(kTlAny) == 0u) continue;
        uint32_t rank[kCentresPerThread], inc = 0u;
#pragma unroll
        for (int h = 0; h < kCentresPerThread; ++h) {
            rank[h] = r[h] ? fetch_inc32(kTlKeys + 4u * key[h]) : 0u;
            // candidate pairs of this item: r(r-1)/2 + r(m-r) per centre
            inc += r[h] ? r[h] * (r[h] - 1) / 2 + r[h] * (m[h] - r[h]) : 0u;
        }
        uint32_t rtot, itot, nne;
        (void)block_excl_scan_at(inc, kTlMisc, &itot);   // its barriers also order the ranks
        const uint32_t bc = tid < 256 ? ld32(kTlKeys + 4u * tid) : 0u;
        const uint32_t bstart = block_excl_scan_at(bc, kTlMisc, &nne);
        if (tid < 256) st32(kTlKeys + 4u * tid, bstart);
        __syncthreads();
#pragma unroll
        for (int h = 0; h < kCentresPerThread; ++h)
            if (r[h]) {   // units: row pairs; m and r packed (both <= the list capacity < 2^16)
                const uint32_t pos = ld32(kTlKeys + 4u * key[h]) + rank[h];
                st32(kSrc + 4u * pos, src[h]);
                st32(kM + 4u * pos, m[h] | (r[h] << 16));
                st32(kRoff + 4u * pos, (r[h] + 1u) >> 1);
            }
        const int nne_u = __builtin_amdgcn_readfirstlane((int)nne);
        __syncthreads();
        // exclusive prefix of the units: thread tid takes compacted centres
        // kCentresPerThread tid, kCentresPerThread tid + 1, ...
        uint32_t rs[kCentresPerThread], rsum = 0u;
#pragma unroll
        for (int h = 0; h < kCentresPerThread; ++h) {
            const int e = kCentresPerThread * tid + h;
            rs[h] = e < nne_u ? ld32(kRoff + 4u * (uint32_t)e) : 0u;
            rsum += rs[h];
        }
        uint32_t rpre = block_excl_scan_at(rsum, kTlMisc, &rtot);
        rtot = __builtin_amdgcn_readfirstlane(rtot);
#pragma unroll
        for (int h = 0; h < kCentresPerThread; ++h) {
            const int e = kCentresPerThread * tid + h;
            if (e < nne_u) st32(kRoff + 4u * (uint32_t)e, rpre);
            rpre += rs[h];
        }
        if (tid == 0) st32(kRoff + 4u * (uint32_t)nne_u, rtot);
        if (rtot == 0) {
            __syncthreads();
            continue;
        }
        if (pending + itot > 0xFFFFFFFFull) {  // keep every uint32 LDS counter exact
            flush(seg);
            zero_hist(G.hb);
            pending = 0;
        }
        pending += itot;
        evaluated += itot;

        // Work units: every row pair is cut into Pp = 2^pp parts of its
        // candidate sequence (run A, then run B), about two units per thread;
        // unit w of centre cl is pair (w - roff[cl] Pp) >> pp, part
        // (w - roff[cl] Pp) & (Pp - 1).
        int pp = 0;
        while (pp < 4 && (rtot << (pp + 1)) <= 2u * kTripletThreads) ++pp;
        const uint32_t U = rtot << pp;
        // chunk table: the centre holding unit 64c, for the waves' first lanes
        const bool chunked = U <= 64u * (uint32_t)kChunkCap;
        __syncthreads();                       // roff complete
        if (chunked) {
#pragma unroll
            for (int h = 0; h < kCentresPerThread; ++h) {
                const int e = kCentresPerThread * tid + h;
                if (e < nne_u) {
                    const uint32_t a = ld32(kRoff + 4u * (uint32_t)e) << pp;
                    const uint32_t b = ld32(kRoff + 4u * (uint32_t)e + 4u) << pp;
                    for (uint32_t c = (a + 63u) >> 6; (c << 6) < b; ++c) st16(kChunkT + 2u * c, (uint32_t)e);
                }
            }
        }
        __syncthreads();

        // the third side is accepted below R3 (R2 unless the third axis is
        // longer); C3 - 1 bounds its components
        const uint32_t R3 = S.R3, R3m1 = S.R3 - 1u;
        constexpr bool kStep = LOOKUP == kLookupStepTable;
        const uint32_t sh = (uint32_t)(kStep ? S.step_sh : S.sh);
        const uint32_t tbits = (uint32_t)(kStep ? S.step_bits : S.tab_bits);
        const int cm1 = S.C3 - 1;
        const int RL = G.rl, nb3 = S.nb3;
        const uint32_t trash = kTlTrash + 4u * (uint32_t)lane;
        // waves take chunks of 64 units from a counter, longest rows first;
        // the next chunk index is fetched while this chunk runs (a wave's
        // last fetch is beyond U and unused)
        uint32_t cix_next = 0;
        if (lane == 0) cix_next = fetch_inc32(kTlNext);
        for (;;) {
            const uint32_t w0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl(cix_next, 0, 64)) * 64u;
            if (w0 >= U) break;
            if (lane == 0) cix_next = fetch_inc32(kTlNext);
            const uint32_t w = w0 + (uint32_t)lane;
            // (compacted) centre of unit w: the wave's first centre from the
            // chunk table, then one step per centre boundary inside the wave's
            // 64 units -- at most 63, since every centre has at least one unit
            int cl;
            if (chunked) {
                const int c0 = (int)ld16(kChunkT + 2u * (w0 >> 6));
                const int ci = c0 + 1 + lane;
                const uint32_t bnd = ci <= nne_u ? ld32(kRoff + 4u * (uint32_t)ci) << pp : 0xffffffffu;
                // mark, in this wave's 64 bytes of the sort buckets (free
                // once the item is set up), the offsets bnd - w0 (1..63, one
                // per centre, in increasing order) at which a centre after c0
                // starts inside the chunk; lane l's centre is c0 plus the marks
                // at offsets <= l.  (Lanes read each other's stores: the
                // wave fences keep the compiler from reordering or forwarding.)
                const uint32_t fl = kTlKeys + 64u * (uint32_t)wave;
                st8(fl + (uint32_t)lane, 0u);
                wave_sync();
                if (bnd <= w0 + 63u) st8(fl + (bnd - w0), 1u);
                wave_sync();
                const uint32_t own = ld8(fl + (uint32_t)lane);
                const uint64_t marks = __ballot(own != 0u);
                cl = c0 + (int)own +
                     (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(marks >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)marks, 0u));
            } else {
                int lo = 0, hi = nne_u - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if ((ld32(kRoff + 4u * (uint32_t)mid) << pp) <= w) lo = mid; else hi = mid - 1;
                }
                cl = lo;
            }
            if (w >= U) continue;
            const uint32_t r0 = ld32(kRoff + 4u * (uint32_t)cl);
            const uint32_t lw = w - (r0 << pp);
            const int jp = (int)(lw >> pp), p = (int)(lw & ((1u << pp) - 1u));
            const uint32_t eoff = ld32(kSrc + 4u * (uint32_t)cl) * ES;   // byte offset of entry J_q
            const uint32_t mr = ld32(kM + 4u * (uint32_t)cl);
            const int mm = (int)(mr & 0xffffu), rr = (int)(mr >> 16);
            // the unit's rows and their runs: row jA over [jA+1, mm), then
            // row jB over [jB+1, mm); this part covers [u0, u1) of the two
            const int jA = jp, jB = rr - 1 - jp;
            const int LA = mm - 1 - jA;
            const int LB = jB > jA ? mm - 1 - jB : 0;
            // Row evaluators: d2, the exact bin, and the increments of a group
            // of 4 candidates (evalg) or of one (eval1) against the current
            // row, which starts as entry v1; second() moves it to entry v2.
            auto with_rows = [&](const E v1, const E v2, auto&& body) {
                // slab index of (b_j, b_k, c) is (b_j - lo0) RL + (b_k - lo0) nb3 + c
                // with RL = (nb - lo0) nb3; entries carry b nb3, and
                // (b_j - lo0) RL = (b_j nb3)(nb - lo0) - lo0 RL
                auto row_base = [&](const E vj) {
                    uint32_t rb = kTlHist +
                                  4u * (uint32_t)(__mul24(Ent<WIDE>::col(vj), nb - lo0) - lo0 * RL - lo0 * nb3);
                    // one opaque value: the address below is then (col + c) << 2
                    // plus rowbase, col read from the entry's high half in place
                    asm volatile("" : "+v"(rb));
                    return rb;
                };
                uint32_t rowbase = row_base(v1), jx, jy = 0, jz;
                if constexpr (WIDE) {
                    jx = (uint32_t)v1.x; jy = (uint32_t)v1.y; jz = (uint32_t)v1.z;
                } else {
                    jx = v1.x; jz = v1.y & 0xffffu;
                }
                auto second = [&]() {
                    rowbase = row_base(v2);
                    if constexpr (WIDE) {
                        jx = (uint32_t)v2.x; jy = (uint32_t)v2.y; jz = (uint32_t)v2.z;
                    } else {
                        jx = v2.x; jz = v2.y & 0xffffu;
                    }
                };
                auto d2 = [&](const E& vk) -> uint32_t {
                    if constexpr (WIDE)
                        return Ent<true>::dist2(vk, (int)jx, (int)jy, (int)jz, cm1);
                    else
                        return Ent<false>::dist2(vk, jx, jz, 0);
                };
                // bin of s; any value for a rejected candidate, whose
                // increment goes to the trash
                auto bin = [&](uint32_t s) -> uint32_t {
                    uint32_t c;
                    if constexpr (kStep) {
                        // one read: the cell's entry carries its bin and the
                        // offset of the threshold inside it
                        c = (ld32(kTlTab + 4u * __builtin_amdgcn_ubfe(s, sh, tbits)) + s) >> sh;
                    } else if constexpr (LOOKUP == kLookupOneStep) {
                        c = ld8(kTlTab + __builtin_amdgcn_ubfe(s, sh, tbits));
                        c += (s >= ld32(kTlThr + 4u + 4u * c)) ? 1u : 0u;
                    } else {
                        const uint32_t sc = min(s, R3m1);
                        c = ld8(kTlTab + (sc >> sh));
                        while (sc >= ld32(kTlThr + 4u + 4u * c)) ++c;
                    }
                    return c;
                };
                // 4 candidates at a time: distances, bins, addresses, then the
                // 4 increments (rejected ones to this lane's trash word)
                auto evalg = [&](const E* v) {
                    uint32_t s[4], a[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) s[u] = d2(v[u]);
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        a[u] = rowbase + 4u * ((uint32_t)Ent<WIDE>::col(v[u]) + bin(s[u]));
                    // keep the address arithmetic unconditional (a select, not a branch)
#pragma unroll
                    for (int u = 0; u < 4; ++u) asm volatile("" : "+v"(a[u]));
#pragma unroll
                    for (int u = 0; u < 4; ++u) inc32(s[u] < R3 ? a[u] : trash);
                };
                auto eval1 = [&](const E& v) {
                    const uint32_t s = d2(v);
                    uint32_t a = rowbase + 4u * ((uint32_t)Ent<WIDE>::col(v) + bin(s));
                    asm volatile("" : "+v"(a));
                    inc32(s < R3 ? a : trash);
                };
                body(evalg, eval1, second);
            };
            auto with_row = [&](const E vj, auto&& body) {
                with_rows(vj, vj, [&](auto& evalg, auto& eval1, auto&) { body(evalg, eval1); });
            };
            // Row j against candidates [k, kend); vj is entry j and ga holds
            // entries [k, k+4) (loaded by the caller, possibly ahead of time).
            // Two register groups in ping-pong, each group's loads issued one
            // group ahead (reads may run up to 7 entries past the list, into
            // the next list or the pool slot's padding, and are never
            // evaluated), then a group of 4 and single candidates.
            auto run = [&](const E vj, E (&ga)[4], int k, int kend) {
                with_row(vj, [&](auto& evalg, auto& eval1) {
                    uint32_t ko = eoff + (uint32_t)k * ES;
                    if (k + 4 <= kend) {
                        E gb[4];
                        for (; k + 8 <= kend; k += 8, ko += 8 * ES) {
                            pool.load4(ko + 4 * ES, gb);
                            evalg(ga);
                            pool.load4(ko + 8 * ES, ga);
                            evalg(gb);
                        }
                        if (k + 4 <= kend) {
                            evalg(ga);
                            k += 4;
                            ko += 4 * ES;
                        }
                    }
                    for (; k < kend; ++k, ko += ES) eval1(pool.load(ko));
                });
            };
            if constexpr (PADDED) {
                // the unit as groups of 4: gA of row jA, then gB of row jB;
                // part p takes groups [g0, g1)
                const int gA = (LA + 3) >> 2, gB = (LB + 3) >> 2, Gt = gA + gB;
                const int g0 = __mul24(p, Gt) >> pp, g1 = __mul24(p + 1, Gt) >> pp;
                const bool hasA = g0 < gA, hasB = g1 > gA;
                const int kA = jA + 1 + 4 * g0, kB = jB + 1 + 4 * (max(g0, gA) - gA);
                E vA{}, gAv[4];
                if (hasA) {
                    vA = pool.load(eoff + (uint32_t)jA * ES);
                    pool.load4(eoff + (uint32_t)kA * ES, gAv);
                }
                // One loop over the part's groups, switching from row jA to
                // row jB after A's last one (koSw), so that a wave's lanes
                // run their A and B groups together instead of every A loop
                // as long as the longest, then every B loop.  A run's last
                // group may reach up to 3 entries past the list, into its pad
                // entries, which every row rejects.  Narrow entries use three
                // register groups, with the loads two groups ahead of the
                // evaluation; the loads past the part (never evaluated) may
                // read 8 entries further, into the next list or the pool
                // slot's padding.  32-bit entries: two groups, one ahead.
                const int nA = hasA ? min(g1, gA) - g0 : 0;
                const int n = g1 - g0;
                if (n <= 0) continue;
                const uint32_t koB = eoff + (uint32_t)kB * ES;
                const uint32_t ko0 = hasA ? eoff + (uint32_t)kA * ES : koB;
                const uint32_t koSw = hasA && hasB ? ko0 + (uint32_t)(nA - 1) * (4u * ES) : 0xffffffffu;
                const E vB = hasB ? pool.load(eoff + (uint32_t)jB * ES) : E{};
                if (!hasA) {
                    pool.load4(koB, gAv);
                    vA = vB;
                }
                with_rows(vA, vB, [&](auto& evalg, auto&, auto& second) {
                    if constexpr (WIDE) {
                        uint32_t ko = ko0;
                        int left = n;
                        E gb[4];
                        for (; left >= 2; left -= 2) {
                            const bool s1 = ko == koSw;
                            const uint32_t k1 = s1 ? koB : ko + 4u * ES;
                            pool.load4(k1, gb);
                            evalg(gAv);
                            if (s1) second();
                            const bool s2 = k1 == koSw;
                            ko = s2 ? koB : k1 + 4u * ES;
                            pool.load4(ko, gAv);
                            evalg(gb);
                            if (s2) second();
                        }
                        if (left) evalg(gAv);
                    } else {
                        auto adv = [&](uint32_t k) -> uint32_t { return k == koSw ? koB : k + 4u * ES; };
                        uint32_t ko = ko0;
                        uint32_t k1 = adv(ko);
                        E gb[4], gc[4];
                        pool.load4(k1, gb);
                        uint32_t k2 = adv(k1);
                        int left = n;
                        for (; left >= 3; left -= 3) {
                            pool.load4(k2, gc);
                            evalg(gAv);
                            if (ko == koSw) second();
                            const uint32_t k3 = adv(k2);
                            pool.load4(k3, gAv);
                            evalg(gb);
                            if (k1 == koSw) second();
                            const uint32_t k4 = adv(k3);
                            pool.load4(k4, gb);
                            evalg(gc);
                            if (k2 == koSw) second();
                            ko = k3; k1 = k4; k2 = adv(k4);
                        }
                        if (left) {
                            evalg(gAv);
                            if (ko == koSw) second();
                            if (left == 2) evalg(gb);
                        }
                    }
                });
                continue;
            }
            const int Lt = LA + LB;
            const int u0 = __mul24(p, Lt) >> pp, u1 = __mul24(p + 1, Lt) >> pp;
            // Both runs' row entries and first groups are loaded before run A
            // starts, so run B begins without a memory round trip (the wide
            // form, short of registers, loads run B's when it starts).  A
            // first group may read up to 3 entries past its run, into the
            // pool padding; they are never evaluated.
            const bool hasA = u0 < LA, hasB = u1 > LA;
            const int kA = jA + 1 + u0, kB = jB + 1 + max(u0, LA) - LA;
            E vA{}, gA[4];
            if (hasA) {
                vA = pool.load(eoff + (uint32_t)jA * ES);
                pool.load4(eoff + (uint32_t)kA * ES, gA);
            }
            if constexpr (!WIDE) {
                E vB{}, gB[4];
                if (hasB) {
                    vB = pool.load(eoff + (uint32_t)jB * ES);
                    pool.load4(eoff + (uint32_t)kB * ES, gB);
                }
                if (hasA) run(vA, gA, kA, jA + 1 + min(u1, LA));
                if (hasB) run(vB, gB, kB, jB + 1 + u1 - LA);
            } else {
                if (hasA) run(vA, gA, kA, jA + 1 + min(u1, LA));
                if (hasB) {
                    E vB = pool.load(eoff + (uint32_t)jB * ES), gB[4];
                    pool.load4(eoff + (uint32_t)kB * ES, gB);
                    run(vB, gB, kB, jB + 1 + u1 - LA);
                }
            }
        }
        __syncthreads();
    }
    if (cur_seg >= 0 && pending) flush(cur_seg);
    if (tid == 0 && evaluated) atomicAdd(A.cand, (unsigned long long)evaluated);
}

// Sum the partial slots of each segment and add them to the output.  The
// thread of slab bin (a, b, c) with a <= b owns half bin (a, b, c): it adds
// the mirror (b, a, c) when b is a slab row too, and writes the output
// (half, or both mirrored full bins), so every output bin has one writer.
// A block first lists the slots of its segment in LDS (in chunks of
// kReduceChunk slots), so each bin sums only those.
constexpr int kReduceChunk = 2048;

__global__ void __launch_bounds__(256) k_reduce(TripletArgs A)
{
    __shared__ int s_idx[kReduceChunk];
    __shared__ int s_n;
    const int seg = blockIdx.y;
    const Seg& G = A.segs[seg];
    if ((int)blockIdx.x * 256 >= G.hb) return;      // whole block past the segment
    const int x = blockIdx.x * 256 + threadIdx.x;
    const Sys& S = A.sys[G.sys];
    const int nb = S.nbins, nb3 = S.nb3, RL = G.rl;
    int a = 0, b = 0, c = 0, xm = 0;
    bool active = x < G.hb;
    if (active) {
        a = G.lo0 + x / RL;
        const int rem = x - (x / RL) * RL;
        b = G.lo0 + rem / nb3;
        c = rem - (rem / nb3) * nb3;
        active = b >= a;
        xm = (b - G.lo0) * RL + (a - G.lo0) * nb3 + c;
    }
    const bool mirror = active && b != a && b < G.lo1;
    const uint32_t used = min(A.ctl->slots_used, (uint32_t)A.max_slots);
    uint64_t sum = 0;
    for (uint32_t base = 0; base < used; base += kReduceChunk) {
        const uint32_t end = min(used, base + (uint32_t)kReduceChunk);
        if (threadIdx.x == 0) s_n = 0;
        __syncthreads();
        for (uint32_t s = base + threadIdx.x; s < end; s += 256)
            if (A.slot_seg[s] == seg) s_idx[atomicAdd(&s_n, 1)] = (int)s;
        __syncthreads();
        const int n = s_n;
        if (active) {
            // four slots per step, their reads in flight together
            int k = 0;
            for (; k + 4 <= n; k += 4) {
                uint32_t v[4], u[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t* sl = A.slots + (size_t)s_idx[k + e] * A.hb_max;
                    v[e] = sl[x];
                    if (mirror) u[e] = sl[xm];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) sum += (uint64_t)v[e] + u[e];
            }
            for (; k < n; ++k) {
                const uint32_t* sl = A.slots + (size_t)s_idx[k] * A.hb_max;
                sum += sl[x];
                if (mirror) sum += sl[xm];
            }
        }
        __syncthreads();
    }
    if (!active || sum == 0) return;
    if (S.tri) {
        S.tri[((size_t)a * nb - (size_t)a * (a - 1) / 2 + (b - a)) * nb3 + c] += sum;
    } else if (S.layout == 0) {
        S.hist[((size_t)a * nb - (size_t)a * (a - 1) / 2 + (b - a)) * nb3 + c] += sum;
    } else if (a == b) {
        S.hist[((size_t)a * nb + a) * nb3 + c] += 2 * sum;
    } else {
        S.hist[((size_t)a * nb + b) * nb3 + c] += sum;
        S.hist[((size_t)b * nb + a) * nb3 + c] += sum;
    }
}

// Triangle-once expansion.  A triangle whose sides fall in bins P, Q (at its
// lowest-ranked atom) and R (opposite) was counted once, at T(lo, hi, R) with
// lo = min(P, Q), hi = max(P, Q).  Seen from each of its three atoms it is
// one unordered pair with the third side opposite, so it owes the half
// histogram one count at each of
//     (lo, hi, R),  (min(lo, R), max(lo, R), hi),  (min(hi, R), max(hi, R), lo).
// Gathered per output bin (x <= y, z), the sources are
//     T(x,y,z) + [x<=z] T(x,z,y) + [x!=y][y<=z] T(y,z,x)
//              + [z<=x] T(z,x,y) + [x!=y][z<=y] T(z,y,x),
// the [x!=y] terms dropping the second copy of a source that coincides with
// the first.  One thread per output bin (full bins (a,b) and (b,a) each
// recompute their half value), adding into the caller's histogram.
__global__ void __launch_bounds__(256) k_expand(const Sys* __restrict__ sys)
{
    const Sys& S = sys[blockIdx.y];
    if (!S.tri) return;
    const int nb = S.nbins;
    const size_t nb3 = (size_t)nb * nb * nb;
    const uint64_t* __restrict__ T = S.tri;
    auto half = [nb](int l, int h, int c) -> size_t {
        return ((size_t)l * nb - (size_t)l * (l - 1) / 2 + (size_t)(h - l)) * nb + c;
    };
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nb3; e += (size_t)gridDim.x * 256) {
        const int a = (int)(e / ((size_t)nb * nb));
        const int b = (int)((e / nb) % nb);
        const int z = (int)(e % nb);
        if (S.layout == 0 && b < a) continue;
        const int x = min(a, b), y = max(a, b);
        uint64_t v = T[half(x, y, z)];
        if (x <= z) v += T[half(x, z, y)];
        if (x != y && y <= z) v += T[half(y, z, x)];
        if (z <= x) v += T[half(z, x, y)];
        if (x != y && z <= y) v += T[half(z, y, x)];
        if (v == 0) continue;
        if (S.layout == 0) S.hist[half(x, y, z)] += v;
        else S.hist[e] += (a == b) ? 2 * v : v;
    }
}

// ------------------------------------------------------------------ launchers
void launch_zero_u32(uint32_t* p, size_t n, hipStream_t s)
{
    if (!n) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}

void launch_cell_count(const Sys* sys, const Job* jobs, int n_jobs, int max_n, hipStream_t s)
{
    hipLaunchKernelGGL(k_cell_count, dim3((max_n + 255) / 256, n_jobs), dim3(256), 0, s, sys, jobs);
}

void launch_cell_scan(const Sys* sys, const Job* jobs, int n_jobs, hipStream_t s)
{
    hipLaunchKernelGGL(k_cell_scan, dim3(n_jobs), dim3(1024), 0, s, sys, jobs);
}

void launch_cell_scatter(const Sys* sys, const Job* jobs, int n_jobs, int max_n, hipStream_t s)
{
    hipLaunchKernelGGL(k_cell_scatter, dim3((max_n + 255) / 256, n_jobs), dim3(256), 0, s, sys, jobs);
}

size_t nbr_build_lds_bytes()
{
    return kThrMax * 4 + 8192 + 256 + (size_t)kBuildWaves * kBufBytes + kBuildWaves * 64 * 4 +
           256 * 4 + (size_t)kBuildWaves * kWaveBufMax * 4 + (size_t)3 * kStageCap * 4;
}

void launch_nbr_build(const Sys* sys, const Job* jobs, int n_jobs, int max_cells, bool wide,
                      bool one_step, int list, unsigned long long* cnt, hipStream_t s)
{
    // enough workgroups per frame to fill the chip, each looping over cells
    // (over the overflow list: a few per frame, most of which find it empty,
    // unless some system leaves all its cells to it)
    const int per_job = list == 1 ? std::min(build_wgs_per_job(n_jobs, max_cells), 8)
                                  : build_wgs_per_job(n_jobs, max_cells);
    const size_t lds = nbr_build_lds_bytes();
    const dim3 g(per_job, n_jobs), b(kBuildThreads);
    const int lm = list ? 1 : 0;
    if (wide) {
        if (one_step) hipLaunchKernelGGL((k_nbr_build<true, true>), g, b, lds, s, sys, jobs, lm, cnt);
        else hipLaunchKernelGGL((k_nbr_build<true, false>), g, b, lds, s, sys, jobs, lm, cnt);
    } else {
        if (one_step) hipLaunchKernelGGL((k_nbr_build<false, true>), g, b, lds, s, sys, jobs, lm, cnt);
        else hipLaunchKernelGGL((k_nbr_build<false, false>), g, b, lds, s, sys, jobs, lm, cnt);
    }
}

size_t nbr_wave_lds_bytes(int stage_cap, bool pairs)
{
    return kWaveShared + (size_t)kWaveBuildWaves * wave_lds(stage_cap, pairs).size;
}

void launch_nbr_wave(const Sys* sys, const Job* jobs, int n_jobs, int n_wgs, int lookup,
                     int stage_cap, bool pairs, unsigned long long* cnt, hipStream_t s)
{
    // wave w of a job's workgroup l (of its n) takes cells 4 l + w + 4 n k
    const size_t lds = nbr_wave_lds_bytes(stage_cap, pairs);
    const int g2 = pairs ? 1 : 0;
    const dim3 g(n_wgs), b(kWaveBuildWaves * 64);
    if (lookup == kLookupStepTable)
        hipLaunchKernelGGL((k_nbr_wave<kLookupStepTable>), g, b, lds, s, sys, jobs, n_jobs, stage_cap, g2, cnt);
    else if (lookup == kLookupOneStep)
        hipLaunchKernelGGL((k_nbr_wave<kLookupOneStep>), g, b, lds, s, sys, jobs, n_jobs, stage_cap, g2, cnt);
    else
        hipLaunchKernelGGL((k_nbr_wave<kLookupSteps>), g, b, lds, s, sys, jobs, n_jobs, stage_cap, g2, cnt);
}

hipError_t set_kernel_lds_limits(size_t triplet_bytes, size_t build_bytes, size_t wave_build_bytes)
{
    const void* trip[9] = {
        (const void*)k_triplet<false, 0, false>, (const void*)k_triplet<false, 1, false>,
        (const void*)k_triplet<false, 2, false>, (const void*)k_triplet<false, 0, true>,
        (const void*)k_triplet<false, 1, true>,  (const void*)k_triplet<false, 2, true>,
        (const void*)k_triplet<true, 0, true>,   (const void*)k_triplet<true, 1, true>,
        (const void*)k_triplet<true, 2, true>};
    hipError_t e;
    for (const void* k : trip) {
        // the triplet kernel addresses LDS from 0: it must have no static LDS
        hipFuncAttributes fa;
        if ((e = hipFuncGetAttributes(&fa, k))) return e;
        if (fa.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;
        if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)triplet_bytes)))
            return e;
    }
    const void* build[4] = {(const void*)k_nbr_build<false, false>, (const void*)k_nbr_build<false, true>,
                            (const void*)k_nbr_build<true, false>, (const void*)k_nbr_build<true, true>};
    for (const void* k : build)
        if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)build_bytes)))
            return e;
    const void* wave[2] = {(const void*)k_nbr_wave<false>, (const void*)k_nbr_wave<true>};
    for (const void* k : wave)
        if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)wave_build_bytes)))
            return e;
    return hipSuccess;
}

void launch_triplet(const TripletArgs& a, bool wide, int lookup, bool padded, int n_wg, hipStream_t s)
{
    const size_t lds = triplet_lds_bytes(a.hb_max, a.cb);
    const dim3 g(n_wg), b(kTripletThreads);
    // wide pad entries are always rejected: the wide form always runs padded
    if (wide) {
        if (lookup == kLookupStepTable) hipLaunchKernelGGL((k_triplet<true, 2, true>), g, b, lds, s, a);
        else if (lookup == kLookupOneStep) hipLaunchKernelGGL((k_triplet<true, 1, true>), g, b, lds, s, a);
        else hipLaunchKernelGGL((k_triplet<true, 0, true>), g, b, lds, s, a);
    } else if (padded) {
        if (lookup == kLookupStepTable) hipLaunchKernelGGL((k_triplet<false, 2, true>), g, b, lds, s, a);
        else if (lookup == kLookupOneStep) hipLaunchKernelGGL((k_triplet<false, 1, true>), g, b, lds, s, a);
        else hipLaunchKernelGGL((k_triplet<false, 0, true>), g, b, lds, s, a);
    } else {
        if (lookup == kLookupStepTable) hipLaunchKernelGGL((k_triplet<false, 2, false>), g, b, lds, s, a);
        else if (lookup == kLookupOneStep) hipLaunchKernelGGL((k_triplet<false, 1, false>), g, b, lds, s, a);
        else hipLaunchKernelGGL((k_triplet<false, 0, false>), g, b, lds, s, a);
    }
}

void launch_reduce(const TripletArgs& a, int max_hb, int n_segs, hipStream_t s)
{
    if (n_segs <= 0) return;
    hipLaunchKernelGGL(k_reduce, dim3((max_hb + 255) / 256, n_segs), dim3(256), 0, s, a);
}

void launch_expand(const Sys* sys, int n_sys, int max_nbins, hipStream_t s)
{
    if (n_sys <= 0) return;
    const size_t nb3 = (size_t)max_nbins * max_nbins * max_nbins;
    size_t blocks = (nb3 + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_expand, dim3((unsigned)blocks, n_sys), dim3(256), 0, s, sys);
}

}  // namespace g3
