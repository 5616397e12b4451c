// Shared definitions between the HIP kernels (g3_kernels.hip) and the host
// runtime (g3_host.cpp) of libg3.  Plain structs only: they are copied to
// device memory as tables.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace g3 {

constexpr int kMaxSlabs = 63;          // r12 slabs per system (slab counts fit one wave)
constexpr int kThrMax = 512;           // threshold table entries (third-side bins + 1)
constexpr int kTripletThreads = 1024;  // threads of the triplet workgroup
constexpr int kCentresPerThread = 2;   // centres a triplet thread sets up per item
constexpr int kListCap = 4096;         // neighbours per centre held by the triplet kernel
// Entries written after every non-empty list: never accepted as a neighbour
// of any row (narrow: components -32768, when the geometry guarantees it;
// wide: 2^30), so the triplet kernel may evaluate a run's last group of 4
// past the list's end instead of a remainder loop.
constexpr int kListPad = 3;
// Centres per triplet pass whose candidate pairs stay below 2^32 whatever the
// lists (each centre has at most kListCap (kListCap - 1) / 2 in a slab).
constexpr int kSafeItemCentres = 512;
static_assert((uint64_t)kSafeItemCentres * kListCap * (kListCap - 1) / 2 <= 0xFFFFFFFFull,
              "a safe pass keeps every uint32 LDS counter exact");
constexpr int kTabBytes = 8192;        // LDS bytes of the bin lookup table
constexpr int kWave = 64;
constexpr int kNbinsMax = 160;         // G3_MAX_NBINS
constexpr int kPoolPad = 8;          // entries after each frame's pool slot that unrolled reads may touch
constexpr int kCursorStride = 32;   // uint32 words between per-frame pool cursors (one 128 B line each)
constexpr int kOvfWord = 1;         // word of a frame's cursor line counting its overflow cells

// Per-frame status bits (one uint32 per frame and system).
constexpr uint32_t kFlagDomain = 1u;   // coordinate outside [0, L)
constexpr uint32_t kFlagPool = 2u;     // neighbour lists exceed the frame's pool slot
constexpr uint32_t kFlagList = 4u;     // one centre exceeds the per-centre capacity
constexpr uint32_t kFlagDense = 8u;    // a list longer than m_safe: recomputed with safe items

// Neighbour entry (minimum-image vector d_ij and its pair bin b):
//  narrow (C <= 32767): x = (dx & 0xffff) | dy << 16, y = (dz & 0xffff) | (b * nbins) << 16
//  wide:                int4 {dx, dy, dz, b * nbins}
// Reference point of cell k (0 <= k < nc <= 1024) on an axis of L < 2^29
// units: the cell's midpoint (2k+1) L / (2 nc), from the width floor(L 2^20 /
// nc) in fixed point, rounded down; within one unit of the exact midpoint.
__host__ __device__ inline uint64_t cell_mid_step(int L, int nc)
{
    return ((uint64_t)L << 20) / (uint64_t)nc;
}
__host__ __device__ inline int cell_mid(uint64_t step, int k)
{
    return (int)(((uint64_t)(2 * k + 1) * step) >> 21);
}

struct Sys {
    // inputs
    const int32_t* frames;   // [F][3][N]
    uint64_t* hist;          // output (added into)
    uint64_t* pair_hist;     // [nbins] ordered pairs per bin (added into), or null
    uint64_t* tri;           // triangle-once mode: [half bins] triangles counted from their
                             // lowest-ranked atom, expanded into hist at the end; null:
                             // every centre's pairs are counted into hist directly
    int32_t F, N;
    int32_t box[3];
    int32_t nc[3];           // cells per axis; 1 means "whole axis, explicit minimum image"
    uint64_t mid_q[3];       // cell width in 2^-20 units (cell_mid_step), for cell_mid
    int32_t ncell;
    int32_t C;               // ceil(rmax): every accepted component satisfies |d| <= C-1
    uint32_t R2;             // thr[nbins]: a pair is accepted iff s < R2
    int32_t C3;              // least C3 with C3^2 >= R3: third-side components |d| <= C3-1
    uint32_t R3;             // thr[nb3]: a third side is accepted iff s < R3
    int32_t nb3;             // third-side bins (nbins..2 nbins); entries carry b * nb3
    int32_t nbins, layout, wide;
    int32_t sh, tab_len;     // bin table: tab[s >> sh] is b(s) or b(s)-1 or lower
    int32_t tab_bits;        // tab_len = 2^tab_bits
    int32_t one_step;        // 1: tab[s >> sh] is b(s) or b(s)-1
    const uint32_t* thr;     // device [nbins + 1]
    const uint8_t* tab;      // device [tab_len]
    // step table (one read per bin): for s < R3 in cell q = s >> step_sh,
    // b(s) = (step[q] + s) >> step_sh; null when no such table of at most
    // kTabBytes / 4 cells exists
    const uint32_t* step;    // device [step_len]
    int32_t step_sh, step_bits, step_len;
    int32_t n_slabs;
    int32_t slab_lo[kMaxSlabs + 1];   // slab q holds rows lo in [slab_lo[q], slab_lo[q+1])
    int32_t list_cap;        // max neighbours per centre
    int32_t pad_ok;          // the pad entries are rejected by every row
    int32_t m_safe;          // longest list for which an item's candidate pairs stay below 2^32
    // scratch (frame f uses base + f * stride; stride 0 = reused every frame)
    int32_t* cell_count;     // [ncell]        stride ncell*cell_mul
    int32_t* cell_start;     // [ncell + 1]
    int32_t* atom_cell;      // [N]
    int32_t* atom_rank;      // [N]
    int32_t* sorted;         // [3][N]
    uint32_t* nbr_off;       // [N]  offset of each centre's list in the frame's pool slot
    uint32_t* nbr_cnt;       // [N]  its length
    uint32_t* cursor;        // [F * kCursorStride]  pool slot fill level (always per frame)
    uint16_t* slab_j;        // [N][n_slabs + 1]  J_q = #entries with bin < slab_lo[q];
                             // a list is partitioned by slab: slab q holds [J_q, J_q+1)
    void* pool;              // entries, 8 or 16 bytes each
    int64_t pool_cap;        // entries per frame slot (the slot stride is pool_cap + kPoolPad)
    int32_t per_frame;       // 1: every frame has its own scratch; 0: reused
    uint32_t* flags;         // [F] (always per frame)
    // per-wave build: the stencil of every cell, relative to the cell's
    // midpoint, fits int16 (pk_ok); cells it leaves to the general build are
    // listed here ([ncell] per frame, count in the frame's cursor line)
    int32_t pk_ok;
    int32_t* ovf_cells;
    uint32_t chunk;          // pool entries a build wave reserves at a time
};

struct Job {
    int32_t sys;
    int32_t frame;
    int32_t wg0;             // per-wave build: this job's first workgroup in its launch
};

// A run of work items of the persistent triplet kernel: one system, one
// r12 slab, frames [frame0, frame0 + n_frames), all centre blocks.
struct Seg {
    int32_t sys;
    int32_t slab;
    int32_t frame0;
    int32_t n_frames;
    int32_t n_blocks;        // centre blocks per frame
    int32_t item_begin;      // first global item index
    int32_t lo0, lo1;        // slab rows
    int32_t hb;              // LDS bins of the slab: (lo1 - lo0) * rl
    int32_t rl;              // bins per slab row: (nbins - lo0) * nbins
    int32_t step;            // items per run handed to a workgroup
    int32_t fetch_begin;     // first run index: runs are numbered in segment order
};

struct Ctl {
    uint32_t next_item;
    uint32_t slots_used;
    uint32_t pad[62];
};

struct TripletArgs {
    const Sys* sys;
    const Seg* segs;
    int32_t n_segs;
    int32_t total_items;
    int32_t n_fetch;         // runs of items (the work counter's range)
    Ctl* ctl;
    uint32_t* slots;         // [max_slots][hb_max]
    int32_t* slot_seg;       // [max_slots]
    int32_t max_slots;
    int32_t hb_max;          // LDS histogram bins
    int32_t cb;              // centres per item
    int32_t tb_max;          // bytes reserved for the bin table
    unsigned long long* cand;  // running count of candidate (centre, {j,k}) pairs evaluated
};

// Triplet kernel LDS: thr (2 KB), bin table, 64 trash words, 32 words of
// scalars, 256 sort buckets, then the histogram slab and per-item centre
// arrays and the work-unit chunk table (uint16, one per 64 units).
constexpr int kChunkCap = 2048;
constexpr uint32_t kTripletLdsFixed = 4 * kThrMax + kTabBytes + 256 + 128 + 1024;
inline size_t triplet_lds_bytes(int hb_max, int cb)
{
    return kTripletLdsFixed + (size_t)hb_max * 4 + (size_t)(3 * cb + 1) * 4 + 2 * kChunkCap;
}

// Neighbour build launch shape: workgroups per frame (each loops over cells),
// waves per workgroup and the pool entries a wave reserves at a time.
constexpr int kBuildWavesPerWG = 8;
constexpr uint32_t kBuildChunk = 2048;     // batched launches (many cells per wave)
constexpr uint32_t kPlainChunk = 256;      // per-frame launches (about one cell per wave)
constexpr int kStageCap = 768;       // stencil atoms staged in LDS per home cell
inline int build_wgs_per_job(int n_jobs, int max_cells)
{
    // about 4 resident workgroups per CU on 256 CUs, all in one round
    int per_job = 1024 / (n_jobs > 0 ? n_jobs : 1);
    if (per_job > max_cells) per_job = max_cells;
    return per_job < 1 ? 1 : per_job;
}

// Per-wave build: 4-wave workgroups (one wave per SIMD, so that as many fit
// as LDS and registers allow), at most seven per CU (the kernel's VGPR
// budget gives seven waves per SIMD).
constexpr size_t kLdsPerCU = 160 * 1024;
constexpr int kWaveBuildWavesPerWG = 4;
constexpr int kWaveBuildMaxWgsPerCU = 7;
inline int wave_wgs_per_cu(size_t lds_bytes)
{
    // LDS is granted in blocks of 512 bytes
    const size_t blocks = (lds_bytes + 511) / 512;
    const int n = (int)(kLdsPerCU / (blocks > 0 ? blocks * 512 : 512));
    return n < 1 ? 1 : (n > kWaveBuildMaxWgsPerCU ? kWaveBuildMaxWgsPerCU : n);
}

// Static scratch for callers that cannot allocate (g3_static.hip): its
// device address on `device` (looked up once per device; the caller makes
// `device` current), and a writer of small tables through kernel arguments.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
constexpr int kPutWords = 760;        // uint32 words per table-writing launch (<= 4 KB of arguments)
void* static_scratch(int device, hipError_t* err);
void launch_put_words(uint32_t* dst, const uint32_t* src, size_t n_words, hipStream_t s);

// Launch wrappers (defined in g3_kernels.hip).
void launch_zero_u32(uint32_t* p, size_t n, hipStream_t s);
void launch_cell_count(const Sys* sys, const Job* jobs, int n_jobs, int max_n, hipStream_t s);
void launch_cell_scan(const Sys* sys, const Job* jobs, int n_jobs, hipStream_t s);
void launch_cell_scatter(const Sys* sys, const Job* jobs, int n_jobs, int max_n, hipStream_t s);
size_t nbr_build_lds_bytes();
// General build over every cell of every job (list 0), or over the cells the
// per-wave build left in each frame's overflow list: a few workgroups per
// frame (list 1), or the full grid when some system leaves all its cells
// there (list 2).
void launch_nbr_build(const Sys* sys, const Job* jobs, int n_jobs, int max_cells, bool wide,
                      bool one_step, int list, unsigned long long* cnt, hipStream_t s);
// Bin lookups of the triplet kernel and the per-wave build: u8 table then
// threshold steps (loop or one step), or the step table.
enum Lookup : int { kLookupSteps = 0, kLookupOneStep = 1, kLookupStepTable = 2 };
// Per-wave build (narrow entries): a wave stages one cell's stencil, at most
// stage_cap atoms, as packed int16 coordinates and builds its centres' lists.
// A 1-D grid of n_wgs workgroups: job j owns workgroups [jobs[j].wg0,
// jobs[j+1].wg0) (the last up to n_wgs).
constexpr int kWaveBuildWaves = kWaveBuildWavesPerWG;
// `pairs`: some system of the launch counts the pair histogram (each wave
// then holds pair counters in LDS).
size_t nbr_wave_lds_bytes(int stage_cap, bool pairs);
void launch_nbr_wave(const Sys* sys, const Job* jobs, int n_jobs, int n_wgs, int lookup,
                     int stage_cap, bool pairs, unsigned long long* cnt, hipStream_t s);
void launch_triplet(const TripletArgs& a, bool wide, int lookup, bool padded, int n_wg, hipStream_t s);
void launch_reduce(const TripletArgs& a, int max_hb, int n_segs, hipStream_t s);
void launch_expand(const Sys* sys, int n_sys, int max_nbins, hipStream_t s);
hipError_t set_kernel_lds_limits(size_t triplet_bytes, size_t build_bytes, size_t wave_build_bytes);

}  // namespace g3
