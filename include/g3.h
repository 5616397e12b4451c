/*
 * g3.h -- C ABI of libg3: the triplet correlation histogram g3(r12, r13, r23)
 * of molecular-simulation frames on AMD Instinct MI355X (gfx950).
 *
 * The quantity is the three-particle correlation function of Sec. 3.3
 * (Eq. 3): for every frame, every centre atom i and every unordered pair
 * {j, k} of other atoms, the three sides r_ij, r_ik and r_jk of the triplet are
 * binned into a 3-D histogram when all three lie below the cutoff.  The third
 * side is taken from the centre's minimum-image neighbour vectors
 * (d_jk = d_ik - d_ij, the "updated positions" of the paper's serial g3
 * logic), with no second minimum image.  Positions are fixed-point integers,
 * bins come from exact integer squared-distance thresholds
 * thr[b] = ceil((b * rmax / nbins)^2), and counts are uint64, so results are
 * exact and reproducible bit for bit.
 *
 * Conventions shared by every entry point
 *   frames   device pointer, int32, layout [n_frames][3][n_atoms] (x row, y row,
 *            z row per frame); every coordinate must satisfy 0 <= x_d < box[d].
 *   box      host array of 3 positive int32 edges of the orthorhombic periodic
 *            box, in the same unit as the coordinates, each <= 2^29.
 *   rmax     cutoff in coordinate units (binary64, used exactly); requires
 *            1 <= rmax <= 46340 and 2*rmax < box[d] on every axis.
 *   nbins    bins per axis, 1..G3_MAX_NBINS; bin width dr = rmax / nbins,
 *            bins half-open [b dr, (b+1) dr), cutoff strict.  The accumulate
 *            calls keep the histogram in LDS slabs of whole rows lo, at most
 *            63 per system, each row holding (nbins - lo) * nbins_third
 *            uint32 counters within the tuning's LDS histogram
 *            (lds_hist_bins): with the default tuning nbins <= 147 when
 *            nbins_third = nbins and <= 116 when nbins_third = 2 nbins
 *            (139 and 110 at 2048 centres per item); a larger nbins makes
 *            them return G3_EINVAL before queuing anything.
 *   layout   G3_HALF: unordered {j,k}, index ((rowoff(lo) + hi - lo) * nbins + c)
 *            with lo = min(b_ij, b_ik), hi = max, c = b_jk and
 *            rowoff(lo) = lo*nbins - lo*(lo-1)/2; nbins*nbins*(nbins+1)/2 bins.
 *            G3_FULL: ordered (j,k), index ((b_ij * nbins + b_ik) * nbins + c);
 *            nbins^3 bins (off-diagonal = half, diagonal lo == hi = 2 x half).
 *   hist     device pointer, uint64, g3_hist_len(nbins, layout) entries.  The
 *            library ADDS into it, so split or resumed runs sum exactly.
 *   pair_hist  optional device pointer (NULL = not wanted), uint64, nbins
 *            entries: the pair histogram behind g2(r) (the paper computes g2
 *            beside g3 in the same pass, Sec. 3.3): for every frame and every
 *            ordered pair (i, j), j != i, with |d_ij| < rmax, entry b(|d_ij|^2)
 *            gains 1 -- the neighbour lists the triplet pass is built from,
 *            counted.  ADDED into with device atomics, so several systems may
 *            share one; it must not overlap any hist.
 *
 * Ownership and ordering: the caller owns frames, hist and all host arrays;
 * the plan owns its device scratch.  Work is queued on the plan's HIP stream
 * and is asynchronous: frames and hist must stay valid and untouched until
 * g3_sync() returns.  A plan is not thread-safe; use one plan per stream.
 * Functions return a status and never throw across the ABI.
 */
#ifndef G3_H
#define G3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define G3_MAX_NBINS 160
#define G3_MAX_RMAX 46340.0

typedef struct g3_plan_s* g3_plan;

typedef enum {
    G3_OK = 0,
    G3_EINVAL = 1,   /* argument outside the documented range */
    G3_EDOMAIN = 2,  /* a coordinate outside [0, box[d]) (reported by g3_sync) */
    G3_ENOMEM = 3,   /* device memory exhausted, or one centre has more
                        neighbours than the plan's per-centre capacity */
    G3_EDEVICE = 4,  /* HIP runtime error */
    G3_EBUSY = 5     /* queued work still running (g3_query) */
} g3_status;

typedef enum { G3_HALF = 0, G3_FULL = 1 } g3_layout;

/* One system of a batch: its own frames, box, cutoff, bins, layout and
 * output histogram (all conventions as above). */
typedef struct {
    const int32_t* frames;
    int32_t n_frames;
    int32_t n_atoms;
    int32_t box[3];
    double rmax;
    int32_t nbins;
    int32_t layout;
    uint64_t* hist;
    uint64_t* pair_hist;     /* optional, may be NULL */
    int32_t nbins_third;     /* bins of the third side (b_jk), same width
                                rmax / nbins: 0 or nbins = third side below
                                rmax; up to 2 nbins = below nbins_third * rmax /
                                nbins.  With rmax = L/4 and 2 nbins this is the
                                paper's geometry (Sec. 3.3: two sides below L/4,
                                the third below L/2).  hist then has
                                g3_hist_len3(nbins, nbins_third, layout) bins,
                                index ((b_ij * nbins + b_ik) * nbins_third + c)
                                (full) or ((rowoff(lo) + hi - lo) * nbins_third
                                + c) (half).  Requires nbins_third * rmax /
                                nbins <= G3_MAX_RMAX; such a system always uses
                                the per-centre enumeration (g3_tuning). */
} g3_system;

/* Tuning knobs of the triplet kernel (chosen by g3_autotune or set by hand).
 * Any value <= 0 means "library default".  None of them changes results. */
typedef struct {
    int32_t lds_hist_bins;   /* uint32 histogram bins held in LDS per workgroup
                                (the r12 slab size); slabs are whole rows lo */
    int32_t centres_per_item;/* centres in one work item of the persistent kernel
                                (at most 2048; a frame with a list longer than
                                fits such items below 2^32 candidate pairs is
                                recomputed with 512-centre items) */
    int32_t wg_per_cu;       /* resident workgroups per compute unit (1 or 2) */
    int32_t per_centre;      /* 1: evaluate every centre's unordered neighbour pairs
                                (the paper's loop, each triangle met at all three
                                atoms); default: meet each triangle once, at its
                                lowest-ranked atom, and expand it exactly into the
                                three histogram entries it owes */
    int32_t slot_limit;      /* partial-histogram slots of one triplet launch; a
                                workgroup whose slab cannot take a slot adds it
                                to the output with 64-bit atomics instead.
                                Default: one per workgroup and segment, up to
                                256 MiB of slots; small values force the atomic
                                path (for tests).  The autotuner keeps it. */
} g3_tuning;

/* Create a plan bound to a HIP stream (hipStream_t passed as void*, NULL =
 * the default stream) on the current device.  Allocates nothing yet. */
g3_status g3_plan_create(g3_plan* out, void* hip_stream);

/* Release the plan and all its device scratch (synchronises its stream). */
void g3_plan_destroy(g3_plan p);

/* Plain form (the paper's per-frame pattern, Sec. 3.3, parallel g3 logic):
 * for each frame one sequence of kernel launches -- cell build, neighbour
 * lists, triplet binning, flush -- on the plan's stream, adding into hist
 * (and into pair_hist unless it is NULL).
 * Returns G3_EINVAL for invalid arguments without queuing any work. */
g3_status g3_accumulate(g3_plan p, const int32_t* frames, int32_t n_frames,
                        int32_t n_atoms, const int32_t box[3], double rmax,
                        int32_t nbins, int32_t layout, uint64_t* hist,
                        uint64_t* pair_hist);

/* Plain form for one described system (all g3_system fields, including
 * pair_hist and nbins_third); otherwise as g3_accumulate. */
g3_status g3_accumulate_system(g3_plan p, const g3_system* system);

/* Batched form: every frame of every system in ONE launch sequence (batched
 * cell and neighbour builds, one persistent triplet kernel pulling work items
 * from a device counter, one flush at the end), replayed as a hipGraph once
 * the same launch signature (shapes and tuning) repeats.  This is the
 * frame x atom flattening of Sec. 3.2's parallel P2 logic (all frames'
 * atoms in one kernel launch instead of a launch per frame, which removes the
 * time between kernel calls), applied to g3 and extended across systems.
 * Systems may differ in size, box, rmax, nbins and layout.  Several systems
 * may not share one hist.  Arguments are checked before anything is queued
 * (G3_EINVAL: a system fails the conventions above, or two systems' hist or
 * pair_hist arrays overlap). */
g3_status g3_accumulate_batch(g3_plan p, const g3_system* systems, int32_t n_systems);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the plain
 * form of g3_accumulate_system (same arguments, same results, one frame at a
 * time on the plan's stream) with every scratch buffer taken from a static
 * device array of G3_NOALLOC_BYTES that the library holds on each GPU it runs
 * on (from module load until the process ends).  It calls no hipMalloc,
 * hipFree or other allocating routine; its tables are written by kernels
 * that take them as arguments.  The caller still owns frames, hist and
 * pair_hist.
 * Limits: one frame's scratch -- about 16 bytes per atom plus 8 bytes per
 * neighbour-list entry with the library's headroom (roughly 100 MiB for
 * N = 65536 at 96 neighbours per atom), plus the bin tables and up to 1/8 of
 * the array for partial histogram slots -- must fit G3_NOALLOC_BYTES, else
 * G3_ENOMEM is returned before anything is queued; at most 65536 frames per
 * call; G3_EDEVICE if the array's address could not be obtained on this
 * device.  Every such call on one GPU shares that GPU's array (it keeps the
 * last call's contents; the library clears what must start at zero): calls
 * from different plans or streams that overlap in time on one GPU race.
 * g3_sync recomputes flagged frames as for g3_accumulate, through the same
 * array; a frame whose neighbour lists overflow even the largest pool that
 * fits it makes g3_sync return G3_ENOMEM. */
#define G3_NOALLOC_BYTES (128u << 20)
g3_status g3_accumulate_noalloc(g3_plan p, const g3_system* system);

/* Wait for the plan's queued work and report asynchronous errors:
 * G3_EDOMAIN if a frame held a coordinate outside the box (such frames add
 * nothing to hist or pair_hist), G3_ENOMEM if a centre exceeded the
 * per-centre neighbour capacity (its frame adds nothing to hist; its pairs
 * are still counted in pair_hist), G3_EDEVICE on a HIP error.  Frames whose
 * neighbour lists overflowed the batched scratch estimate, or were too long
 * for the tuning's work items to keep every 32-bit counter exact, are
 * recomputed here through the plain path (with 512-centre items) before
 * returning, so they are never lost or miscounted. */
g3_status g3_sync(g3_plan p);

/* Completion of one call without waiting for the rest of the stream (for
 * serving loops that keep several calls in flight).  Every successful
 * g3_accumulate, g3_accumulate_system and g3_accumulate_batch call gets a
 * ticket, numbered 1, 2, ... per plan; g3_last_ticket returns the latest
 * (0 before the first).  g3_ticket_query never blocks:
 *   G3_EBUSY  the call's kernels are still running;
 *   G3_OK     they have finished, and *final says whether every histogram the
 *             call added into now holds its final counts (1), or whether
 *             g3_sync must run first (0: a frame of the call is to be
 *             recomputed, or an error is to be reported);
 *   G3_EINVAL no such ticket.
 * Every ticket issued before a g3_sync is final once it returns.  A copy of
 * a histogram taken after a ticket reports final = 1 holds the call's
 * counts; if g3_sync had to run, copy it again after g3_sync. */
g3_status g3_last_ticket(g3_plan p, uint64_t* ticket);
g3_status g3_ticket_query(g3_plan p, uint64_t ticket, int32_t* final);

/* Non-blocking: G3_OK if all work queued on the plan's stream has finished
 * (g3_sync will then not wait), G3_EBUSY if some is still running. */
g3_status g3_query(g3_plan p);

/* Histogram length for (nbins, layout); 0 if invalid. */
size_t g3_hist_len(int32_t nbins, int32_t layout);

/* Histogram length with nbins_third third-side bins (nbins..2 nbins). */
size_t g3_hist_len3(int32_t nbins, int32_t nbins_third, int32_t layout);

/* Host-side validation of one system's arguments (no device work). */
g3_status g3_check_args(int32_t n_atoms, const int32_t box[3], double rmax,
                        int32_t nbins, int32_t layout);

/* Exact thresholds thr[b] = ceil((b * rmax / nbins)^2), b = 0..nbins, written
 * to the host array thr (nbins + 1 entries). */
g3_status g3_thresholds(double rmax, int32_t nbins, uint32_t* thr);

/* Ideal-gas normalisation (Eq. 3 with U = 0; host, fp64):
 *   g3 = H / E,  E = n_frames * N (N-1)(N-2) / V^2 * W(a,b,c)   (full layout),
 * with E halved on the half-layout diagonal and g3 = 0 where W = 0.
 * W(a,b,c) = 8 pi^2 \int\int\int r s t 1[|r-s| <= t <= r+s] over the bin box is
 * evaluated exactly: dr^6 pi^2 times a rational number obtained from the
 * closed-form volume of ball-ball lens intersections.  hist and g3_out are
 * host arrays of g3_hist_len(nbins, layout) entries. */
g3_status g3_normalize(const uint64_t* hist, int32_t layout, int32_t nbins, double rmax,
                       int64_t n_frames, int32_t n_atoms, const int32_t box[3],
                       double* g3_out);

/* g3_normalize for a histogram with nbins_third third-side bins (the same
 * formula; W(a, b, c) for c up to nbins_third - 1). */
g3_status g3_normalize3(const uint64_t* hist, int32_t layout, int32_t nbins,
                        int32_t nbins_third, double rmax, int64_t n_frames,
                        int32_t n_atoms, const int32_t box[3], double* g3_out);

/* Ideal-gas normalisation of the pair histogram (host, fp64):
 *   g2[b] = H2[b] / E2[b],  E2[b] = n_frames * N (N-1) / V * 4 pi/3 (r_{b+1}^3 - r_b^3),
 * r_b = b * rmax / nbins (ordered pairs, as pair_hist counts them).  Both
 * arrays hold nbins entries. */
g3_status g3_normalize_pairs(const uint64_t* pair_hist, int32_t nbins, double rmax,
                             int64_t n_frames, int32_t n_atoms, const int32_t box[3],
                             double* g2_out);

/* Superposition ratio (Kirkwood's approximation g3 ~ g2 g2 g2 tested bin by
 * bin; the angle-resolved motivation of Sec. 3.3): out[x] = g3[x] /
 * (g2[a] g2[b] g2[c]) for the bin (a, b, c) at index x of the layout, 0 where
 * the product is 0.  g3 and out: host, g3_hist_len(nbins, layout) doubles
 * (e.g. from g3_normalize); g2: host, nbins doubles (g3_normalize_pairs). */
g3_status g3_superposition(const double* g3, int32_t layout, int32_t nbins, const double* g2,
                           double* out);

/* Isosceles slice g3(r, r, theta): both sides at the apex in bin a, third
 * side in bin c = 0..nbins-1.  value[c] = g3(a, a, c) (either layout);
 * theta[c] = the apex angle, in radians, of the triangle with both sides at
 * the centre of bin a and the third side at the centre of bin c,
 * 2 asin((c + 1/2) / (2 (a + 1/2))), or -1 where that third side exceeds
 * twice the other two (no triangle).  Host arrays of nbins doubles. */
g3_status g3_isosceles(const double* g3, int32_t layout, int32_t nbins, int32_t a,
                       double* theta, double* value);

/* W(a,b,c) for all bins (full layout, nbins^3 doubles, host). */
g3_status g3_ideal_volume(int32_t nbins, double rmax, double* W_out);

/* Tuning: set (copied) or read the plan's knobs. */
g3_status g3_set_tuning(g3_plan p, const g3_tuning* t);
g3_status g3_get_tuning(g3_plan p, g3_tuning* t);

/* Autotuner (the batched form's tile and slab choice): runs the batched form
 * on the given systems into internal scratch histograms (the systems' hist
 * pointers are ignored and never written) over a grid of tunings -- resident
 * workgroups per CU, centres per work item, LDS histogram size (which sets
 * the r12 slab boundaries) -- checks that every tuning yields the identical
 * histogram (G3_EDEVICE if not), keeps the fastest in the plan, caches it
 * under a signature of the workload (entry format, nbins, layout, N and
 * neighbour-count buckets, frames) and returns it in *best (may be NULL).
 * A repeated call with the same signature returns the cached tuning at once.
 * Synchronises the plan's stream. */
g3_status g3_autotune(g3_plan p, const g3_system* systems, int32_t n_systems,
                      g3_tuning* best);

/* Timing of the triplet-kernel launches on the plan's stream since the last
 * g3_kernel_time_reset(p, 1), measured with HIP events (milliseconds per
 * launch, averaged) and the number of launches.  While timing is enabled the
 * batched form launches its kernels directly (no graph replay), so that the
 * events bracket them. */
g3_status g3_kernel_time(g3_plan p, double* avg_ms, int64_t* n_launches);
g3_status g3_kernel_time_reset(g3_plan p, int32_t enable);

/* The same for one stage of the path: G3_STAGE_TRIPLET (triplet binning,
 * = g3_kernel_time), G3_STAGE_NEIGHBOURS (the neighbour build: the per-wave
 * build and the general build over the cells it leaves, one interval),
 * G3_STAGE_CELLS (counting sort into cells). */
enum { G3_STAGE_TRIPLET = 0, G3_STAGE_NEIGHBOURS = 1, G3_STAGE_CELLS = 2 };
g3_status g3_stage_time(g3_plan p, int32_t stage, double* avg_ms, int64_t* n_launches);

/* Work of the neighbour builds since the last g3_kernel_time_reset:
 * candidates = (centre, stencil atom) pairs whose distance was tested (the
 * triangle-once lists test only atoms ranked above the centre), neighbours =
 * entries written to the lists (pairs closer than rmax).  Synchronises the
 * plan's stream. */
g3_status g3_build_counts(g3_plan p, uint64_t* candidates, uint64_t* neighbours);

/* Candidate pairs evaluated by the triplet kernel since the last
 * g3_kernel_time_reset: one per (centre i, unordered {j,k}) with both j and k
 * within rmax of i -- the pairs whose third side the method must test.
 * Synchronises the plan's stream. */
g3_status g3_candidates(g3_plan p, uint64_t* n);

/* Measured LDS rates of the current device, the ceilings behind the triplet
 * kernel's roofline (its LDS work per candidate pair is one bin-table read
 * and one histogram increment).  One 1024-thread workgroup per compute unit,
 * each lane cycling through 16 word addresses in a table of `words` uint32
 * words of LDS (1..36864; at least 1024 for pattern 0):
 *   0  ds_add_u32 on the lane's own word (no bank conflict: the trash words
 *      rejected candidates add to);
 *   1  ds_add_u32 at uniformly random words (histogram increments);
 *   2  ds_read_b32 at uniformly random words (bin-table reads);
 *   3  one random read and one random add per step (counted as 2 operations).
 * *lane_ops_per_s = lane operations per second over the whole device, the
 * best of three timed launches after one warm-up.  Synchronous; allocates
 * and frees a small device buffer. */
g3_status g3_lds_rate(int32_t pattern, int32_t words, double* lane_ops_per_s);

const char* g3_strerror(g3_status s);

#ifdef __cplusplus
}
#endif
#endif /* G3_H */
