// Host-side check of the bin lookup tables built by the runtime (compiled
// with the runtime's source and stub launchers; no GPU).  For every value
// s < R3 of each geometry below, against b(s) = the largest b < nb3 with
// thr[b] <= s:
//   * the u8 table gives a lower bound, within one step when one_step is set;
//   * the step table, when built, gives b(s) exactly.
// Then the pad entries after each neighbour list: where the host lets the
// triplet kernel read them, no row accepts them.  Then the per-wave build's
// int16 staging: wherever the host sets pk_ok, every coordinate of a cell's
// 3 x 3 x 3 stencil (periodic shift applied) minus the kernel's midpoint
// reference fits int16, and the sentinel atoms are rejected by every centre.
// Then the per-wave build's grid over the jobs of a launch, the triplet
// kernel's runs of items, a small batch's segment order and a batch's
// scratch layout.
// Exit status: the number of geometries with a failure.
#include "../paper_1708_08619_amd/csrc/g3_host.cpp"

namespace g3 {
void launch_zero_u32(uint32_t*, size_t, hipStream_t) {}
void launch_cell_count(const Sys*, const Job*, int, int, hipStream_t) {}
void launch_cell_scan(const Sys*, const Job*, int, hipStream_t) {}
void launch_cell_scatter(const Sys*, const Job*, int, int, hipStream_t) {}
size_t nbr_build_lds_bytes() { return 0; }
void launch_nbr_build(const Sys*, const Job*, int, int, bool, bool, int, unsigned long long*, hipStream_t) {}
size_t nbr_wave_lds_bytes(int, bool) { return 0; }
void launch_nbr_wave(const Sys*, const Job*, int, int, int, int, bool, unsigned long long*, hipStream_t) {}
void launch_triplet(const TripletArgs&, bool, int, bool, int, hipStream_t) {}
void launch_reduce(const TripletArgs&, int, int, hipStream_t) {}
void launch_expand(const Sys*, int, int, hipStream_t) {}
hipError_t set_kernel_lds_limits(size_t, size_t, size_t) { return hipSuccess; }
void* static_scratch(int, hipError_t* e) { *e = hipErrorNotSupported; return nullptr; }
void launch_put_words(uint32_t*, const uint32_t*, size_t, hipStream_t) {}
}  // namespace g3

int main()
{
    // rmax in coordinate units, pair bins, third-side bins
    struct Case { double rmax; int nb, nb3; } cases[] = {
        {3.0 * 4096, 60, 60},   {2.5 * 4096, 50, 50},   {2.0 * 4096, 40, 40},
        {0.6 * 65536, 60, 60},  {7.0, 7, 7},            {1000.5, 13, 26},
        {3.0 * 4096, 60, 120},  {23170.0, 160, 160},    {100.0, 1, 1},
        {1.0, 1, 2},            {33.3, 30, 30},         {12345.678, 77, 77},
        {40000.0, 45, 90},      {5000.0, 150, 300},     {2.5 * 4096, 50, 100}};
    int failed = 0, with_step = 0;
    for (const Case& c : cases) {
        Geometry g;
        g.nbins = c.nb;
        g.nb3 = c.nb3;
        plan_bins(g, c.rmax);
        uint64_t bad_tab = 0, bad_step = 0;
        int b = 0;
        const uint32_t qmask = (1u << g.step_bits) - 1u;
        for (uint64_t s = 0; s < g.R3; ++s) {
            while (b + 1 < g.nb3 && s >= g.thr[b + 1]) ++b;
            const int t = g.tab[(size_t)(s >> g.sh)];
            if (t > b || (g.one_step && b - t > 1)) ++bad_tab;
            if (g.step_ok) {
                const uint32_t e = g.step[(uint32_t)(s >> g.step_sh) & qmask];
                if (((e + (uint32_t)s) >> g.step_sh) != (uint32_t)b) ++bad_step;
            }
        }
        with_step += g.step_ok;
        std::printf("rmax %.3f nbins %d nb3 %d: R3 %u one_step %d step_table %d (%zu cells of 2^%d) "
                    "bad %llu %llu\n", c.rmax, c.nb, c.nb3, g.R3, g.one_step, g.step_ok, g.step.size(),
                    g.step_sh, (unsigned long long)bad_tab, (unsigned long long)bad_step);
        failed += (bad_tab || bad_step) ? 1 : 0;
    }
    // the benchmark-like geometries must get the step table
    if (with_step < 8) ++failed;

    // Pad entries (components -32768): where the host lets the triplet kernel
    // read them, every row within the pair cutoff must reject them, in the
    // kernel's arithmetic (saturated 16-bit differences, squares summed and
    // clamped to 2^31 - 1).  Rows on a grid over [-(C-1), C-1]^3, extremes
    // included.
    struct Pad { double rmax; int nb, nb3; bool padded; } pads[] = {
        {3.0 * 4096, 60, 60, true}, {15000.0, 12, 24, true}, {15100.0, 10, 20, true},
        {16000.0, 10, 20, false}, {30000.0, 20, 20, false}, {39321.6, 60, 60, true}};
    for (const Pad& c : pads) {
        Geometry g;
        g.nbins = c.nb;
        g.nb3 = c.nb3;
        g.C = (int)std::ceil(c.rmax);
        plan_bins(g, c.rmax);
        g.wide = g.C3 > 32767 ? 1 : 0;
        const bool padded = pads_rejected(g);
        uint64_t accepted = 0, rows = 0;
        if (padded && !g.wide) {
            auto sat = [](int64_t v) { return v < -32768 ? -32768 : (v > 32767 ? 32767 : v); };
            const int K = 40;
            for (int a = 0; a <= K; ++a)
                for (int b = 0; b <= K; ++b)
                    for (int e = 0; e <= K; ++e) {
                        const int64_t m = g.C - 1;
                        const int64_t jx = -m + 2 * m * a / K, jy = -m + 2 * m * b / K, jz = -m + 2 * m * e / K;
                        if ((uint64_t)(jx * jx + jy * jy + jz * jz) >= g.R2) continue;   // not a row
                        ++rows;
                        const int64_t dx = sat(-32768 - jx), dy = sat(-32768 - jy), dz = sat(-32768 - jz);
                        const int64_t s = std::min<int64_t>(dx * dx + dy * dy + dz * dz, 0x7fffffff);
                        if ((uint64_t)s < g.R3) ++accepted;
                    }
        }
        std::printf("pads: rmax %.1f nb3 %d wide %d padded %d (expected %d): %llu rows, %llu accept a pad\n",
                    c.rmax, c.nb3, g.wide, padded ? 1 : 0, c.padded ? 1 : 0, (unsigned long long)rows,
                    (unsigned long long)accepted);
        if (padded != c.padded || accepted) ++failed;
    }

    // Per-wave build: for boxes and cutoffs around the bound, every cell k of
    // an axis with cells k-1, k, k+1 (wrapped, shifted by the box) staged
    // relative to the reference the kernel uses.  A cell k' holds the
    // integers x with floor(x nc / L) = k'.
    struct Ax { int L; double rmax; } axes[] = {
        {174356, 12288.0}, {28016, 10240.0}, {65600, 21000.0}, {65536, 21844.0}, {70000, 23000.0},
        {100003, 20000.0}, {43000, 14300.0}, {2000000, 21840.0}, {1000, 300.0}, {90, 29.0},
        {65490, 21800.0}, {65520, 21800.0}};
    int staged_ok = 0;
    for (const Ax& a : axes) {
        Geometry g;
        g.N = 1 << 20;
        g.nbins = 10;
        g.nb3 = 10;
        g.box[0] = g.box[1] = g.box[2] = a.L;
        g.C = (int)std::ceil(a.rmax);
        plan_bins(g, a.rmax);
        g.wide = g.C3 > 32767 ? 1 : 0;
        plan_cells(g);
        g.pk_ok = !g.wide && g.C <= 32767;
        for (int d = 0; d < 3; ++d) {
            const double w = (double)g.box[d] / (double)g.nc[d];
            if (g.nc[d] < 3 || !(1.5 * w + 8.0 <= 32767.0)) g.pk_ok = 0;
        }
        const int nc = g.nc[0], L = a.L;
        int64_t worst = 0, home = 0;
        bool bad = false;
        if (g.pk_ok) {
            auto lo_of = [&](int64_t k) { return (k * L + nc - 1) / nc; };   // least x in cell k
            for (int k = 0; k < nc; ++k) {
                const int ref = cell_mid(cell_mid_step(L, nc), k);
                for (int o = -1; o <= 1; ++o) {
                    int kk = k + o, shift = 0;
                    if (kk < 0) { kk += nc; shift = -L; } else if (kk >= nc) { kk -= nc; shift = L; }
                    const int64_t x0 = lo_of(kk), x1 = lo_of(kk + 1) - 1;
                    for (int64_t x : {x0, x1}) {
                        if ((x * nc) / L != kk) bad = true;     // the cell bounds themselves
                        const int64_t rel = x + shift - ref;
                        worst = std::max<int64_t>(worst, rel < 0 ? -rel : rel);
                        if (o == 0) home = std::max<int64_t>(home, rel < 0 ? -rel : rel);
                    }
                }
            }
            // sentinel -32768 against any centre of the home cell: at least
            // 32768 - |c| per component (saturation only raises it)
            const int64_t dmin = 32768 - std::min<int64_t>(home, 32767);
            const int64_t s = std::min<int64_t>(3 * dmin * dmin, 0x7fffffff);
            if (worst > 32767 || (uint64_t)s < g.R2) bad = true;
            staged_ok += 1;
        }
        std::printf("stage: L %d rmax %.1f cells %d pk_ok %d worst |rel| %lld (home %lld) %s\n", L, a.rmax, nc,
                    g.pk_ok, (long long)worst, (long long)home, bad ? "FAIL" : "ok");
        if (bad) ++failed;
    }
    if (staged_ok < 6) ++failed;     // the benchmark-like axes must qualify

    // Per-wave build grid: each job's workgroups start where the previous
    // job's end (the kernel finds its job by binary search over them), every
    // job has at least one and at most one per 4 cells, and a launch has about
    // four rounds of resident workgroups at most, or more to keep at most 16
    // cells in a wave, in whole rounds (one round at least unless that would
    // put fewer than one cell in a wave).
    struct GridCase { std::vector<int> cells; int frames; } grids[] = {
        {{2744}, 50}, {{2744}, 1}, {{1331, 216, 729, 27, 64, 1000, 343, 512}, 8},
        {{1}, 1}, {{3}, 3}, {{161874}, 1}, {{8, 8000000}, 2}};
    for (const GridCase& gc : grids) {
        std::vector<Prepared> ps(gc.cells.size());
        for (size_t k = 0; k < ps.size(); ++k) ps[k].g.ncell = gc.cells[k];
        std::vector<Job> jobs;
        for (size_t k = 0; k < ps.size(); ++k)
            for (int f = 0; f < gc.frames; ++f) jobs.push_back({(int)k, f, -1});
        BuildPlan bp;
        bp.wave = true;
        bp.cap = 480;
        const int n_cu = 256;
        const int total = plan_wave_grid(jobs.data(), (int)jobs.size(), ps, bp, n_cu);
        const int64_t resident = (int64_t)n_cu * wave_wgs_per_cu(nbr_wave_lds_bytes(bp.cap, bp.pairs));
        int64_t cells = 0;
        bool bad = jobs.empty() || jobs[0].wg0 != 0;
        for (size_t j = 0; j < jobs.size(); ++j) {
            const int nc = ps[jobs[j].sys].g.ncell;
            cells += nc;
            const int end = j + 1 < jobs.size() ? jobs[j + 1].wg0 : total;
            const int w = end - jobs[j].wg0;
            if (w < 1 || w > (nc + kWaveBuildWaves - 1) / kWaveBuildWaves) bad = true;
        }
        // at most about four rounds, or 16 cells per wave, in whole rounds
        // (one more round at most; each job's count is rounded up)
        if ((int64_t)total > std::max<int64_t>(4 * resident, cells / (16 * kWaveBuildWaves) + 1) + resident +
                                 (int64_t)jobs.size())
            bad = true;
        // no wave with more than 16 cells
        for (size_t j = 0; j < jobs.size(); ++j) {
            const int end = j + 1 < jobs.size() ? jobs[j + 1].wg0 : total;
            const int64_t per_wave = (ps[jobs[j].sys].g.ncell + (int64_t)(end - jobs[j].wg0) * kWaveBuildWaves - 1) /
                                     ((int64_t)(end - jobs[j].wg0) * kWaveBuildWaves);
            if (per_wave > 16) bad = true;
        }
        // at least one round, or one cell per wave everywhere
        const int64_t one_cell = [&] {
            int64_t t = 0;
            for (const Job& jb : jobs) t += (ps[jb.sys].g.ncell + kWaveBuildWaves - 1) / kWaveBuildWaves;
            return t;
        }();
        if ((int64_t)total < std::min<int64_t>(resident, one_cell)) bad = true;
        std::printf("wave grid: %zu jobs, %lld cells -> %d workgroups (resident %lld) %s\n", jobs.size(),
                    (long long)cells, total, (long long)resident, bad ? "FAIL" : "ok");
        if (bad) ++failed;
    }

    // Runs of items for the triplet kernel: replaying the kernel's mapping
    // (forward scan over segments by first run, item = start + run * step),
    // every item of every segment is handed out exactly once, no run leaves
    // its segment, runs are 1 to 16 items, and a segment with at least one
    // item per workgroup keeps runs of one.
    struct RunCase { std::vector<int> seg_items; int n_wg; } runs[] = {
        {{24, 24, 24, 5, 1, 300, 3}, 256}, {{1600, 1600, 1600, 1600, 1600}, 256},
        {std::vector<int>(400, 24), 256}, {std::vector<int>(1500, 40), 256}, {{7}, 256}, {{100, 2, 9}, 4}};
    for (const RunCase& rc : runs) {
        std::vector<Seg> segs;
        int total = 0;
        for (int k : rc.seg_items) {
            Seg sg{};
            sg.item_begin = total;
            segs.push_back(sg);
            total += k;
        }
        const int n_fetch = plan_runs(segs, total, rc.n_wg);
        std::vector<int> seen(total, 0);
        bool bad = false;
        int q = 0, max_step = 0;
        for (int f = 0; f < n_fetch; ++f) {
            while (q + 1 < (int)segs.size() && segs[q + 1].fetch_begin <= f) ++q;
            const int end = q + 1 < (int)segs.size() ? segs[q + 1].item_begin : total;
            const int item = segs[q].item_begin + (f - segs[q].fetch_begin) * segs[q].step;
            const int n = std::min(segs[q].step, end - item);
            if (item < segs[q].item_begin || n < 1) { bad = true; break; }
            for (int i = item; i < item + n; ++i) ++seen[i];
        }
        for (size_t k = 0; k < segs.size(); ++k) {
            max_step = std::max(max_step, segs[k].step);
            if (segs[k].step < 1 || segs[k].step > 16) bad = true;
            if (rc.seg_items[k] >= rc.n_wg && segs[k].step != 1) bad = true;
        }
        for (int v : seen) if (v != 1) bad = true;
        std::printf("runs: %zu segments, %d items -> %d runs (longest %d) %s\n", segs.size(), total, n_fetch,
                    max_step, bad ? "FAIL" : "ok");
        if (bad) ++failed;
    }

    // Segment order of a small batch: every segment kept, items numbered
    // contiguously in the new order, and within one system (same density and
    // cutoff) an outer slab (more rows beyond it) before an inner one whose
    // rows are fewer -- checked on the benchmark-like slabs (rows from 0, 8,
    // 17, 28, 44 of 60), where the estimate ranks slab 3 and 4 first.
    {
        std::vector<Prepared> ps(3);
        const int Ns[3] = {65536, 4096, 20000};
        for (int k = 0; k < 3; ++k) {
            Prepared& P = ps[k];
            P.g.N = Ns[k];
            P.g.nbins = 60;
            P.g.nb3 = 60;
            const int L = (int)std::lround(std::cbrt((double)Ns[k] / 0.85) * 4096.0);
            P.g.box[0] = P.g.box[1] = P.g.box[2] = L;
            P.in.rmax = 3.0 * 4096;
            P.tri_once = true;
            P.g.slab_lo = {0, 8, 17, 28, 44, 60};
        }
        std::vector<Seg> segs;
        int items = 0;
        for (int k = 0; k < 3; ++k) add_segments(ps[k], k, 0, 5, 2048, segs, items);
        const size_t n_before = segs.size();
        order_segments(segs, ps, 2048);
        bool bad = segs.size() != n_before;
        int it = 0;
        for (const Seg& sg : segs) {
            if (sg.item_begin != it) bad = true;
            it += sg.n_blocks * sg.n_frames;
        }
        if (it != items) bad = true;
        // the first segment of each system is one of its two outer slabs,
        // its last one the innermost
        for (int k = 0; k < 3; ++k) {
            int first = -1, last = -1;
            for (const Seg& sg : segs)
                if (sg.sys == k) {
                    if (first < 0) first = sg.slab;
                    last = sg.slab;
                }
            if (first < 3 || last != 0) bad = true;
        }
        std::printf("segment order: %zu segments, %d items %s\n", segs.size(), items, bad ? "FAIL" : "ok");
        if (bad) ++failed;
    }

    // A batch's scratch layout: systems prepared with the shared bin-table
    // cache get the same tables as without it; no two regions overlap except
    // the tables of systems with the same (rmax, nbins, nbins_third), which
    // are one copy; the block cleared by one fill holds every system's cell
    // counts and pool cursors and nothing else.
    {
        struct Spec { int N, F; double rmax; int nb, nb3, layout; };
        const Spec specs[] = {{4000, 3, 3.0 * 4096, 60, 60, 0}, {9000, 1, 2.5 * 4096, 50, 50, 1},
                              {4000, 2, 3.0 * 4096, 60, 60, 1}, {1500, 4, 2.5 * 4096, 50, 100, 1},
                              {30000, 2, 3.0 * 4096, 60, 60, 0}, {2500, 1, 2.5 * 4096, 50, 50, 0},
                              {700, 5, 2.5 * 4096, 50, 100, 1}, {5000, 2, 2.0 * 4096, 40, 40, 0}};
        std::vector<Prepared> ps;
        BinCache cache;
        bool bad = false;
        static int32_t dummy_frames[1];
        static uint64_t dummy_hist[1];
        for (const Spec& sp : specs) {
            g3_system in{};
            in.frames = dummy_frames;
            in.hist = dummy_hist;
            in.n_frames = sp.F;
            in.n_atoms = sp.N;
            const int L = (int)std::lround(std::cbrt((double)sp.N / 0.85) * 4096.0);
            in.box[0] = in.box[1] = in.box[2] = L;
            in.rmax = sp.rmax;
            in.nbins = sp.nb;
            in.nbins_third = sp.nb3 == sp.nb ? 0 : sp.nb3;
            in.layout = sp.layout;
            Prepared P, Q;
            if (prepare(in, 30784, P, &cache) != G3_OK || prepare(in, 30784, Q) != G3_OK) {
                bad = true;
                continue;
            }
            if (P.g.thr != Q.g.thr || P.g.tab != Q.g.tab || P.g.step != Q.g.step || P.g.sh != Q.g.sh ||
                P.g.step_sh != Q.g.step_sh || P.g.step_ok != Q.g.step_ok || P.g.one_step != Q.g.one_step ||
                P.g.R2 != Q.g.R2 || P.g.R3 != Q.g.R3 || P.g.C3 != Q.g.C3 || P.g.tab_bits != Q.g.tab_bits)
                bad = true;
            ps.push_back(std::move(P));
        }
        const size_t total = layout_scratch(ps, true, false, 0, true, 256);
        struct Region { size_t b, e; int sys; int kind; };
        std::vector<Region> rs;
        auto add = [&](size_t b, size_t n, int k, int kind) { if (n) rs.push_back({b, b + n, k, kind}); };
        for (int k = 0; k < (int)ps.size(); ++k) {
            const Prepared& P = ps[k];
            const size_t F = (size_t)P.in.n_frames, N = (size_t)P.g.N, C = (size_t)P.g.ncell;
            const size_t S = P.g.slab_lo.size() - 1;
            add(P.off_cell_count, F * C * 4, k, 0);
            add(P.off_cursor, F * kCursorStride * 4, k, 0);
            add(P.off_cell_start, F * (C + 1) * 4, k, 1);
            add(P.off_atom_cell, F * N * 4, k, 1);
            add(P.off_atom_rank, F * N * 4, k, 1);
            add(P.off_sorted, F * 3 * N * 4, k, 1);
            add(P.off_nbr_off, F * N * 4, k, 1);
            add(P.off_nbr_cnt, F * N * 4, k, 1);
            add(P.off_slab_j, F * N * (S + 1) * 2, k, 1);
            add(P.off_ovf, F * C * 4, k, 1);
            add(P.off_pool, F * (size_t)(P.pool_cap + kPoolPad) * (P.g.wide ? 16 : 8), k, 1);
            if (P.tri_once) add(P.off_tri, g3_hist_len(P.g.nbins, G3_HALF) * 8, k, 1);
            bool shared = false;
            for (int j = 0; j < k; ++j) {
                const bool same = ps[j].in.rmax == P.in.rmax && ps[j].g.nbins == P.g.nbins &&
                                  ps[j].g.nb3 == P.g.nb3;
                const bool same_off = ps[j].off_thr == P.off_thr;
                if (same != same_off) bad = true;
                if (same) {
                    shared = true;
                    if (ps[j].off_tab != P.off_tab || ps[j].off_step != P.off_step) bad = true;
                }
            }
            if (!shared) {
                add(P.off_thr, (P.g.nb3 + 1) * 4, k, 2);
                add(P.off_tab, (size_t)P.g.tab_len, k, 2);
                add(P.off_step, P.g.step.size() * 4, k, 2);
            }
        }
        for (size_t i = 0; i < rs.size(); ++i) {
            if (rs[i].e > total) bad = true;
            for (size_t j = i + 1; j < rs.size(); ++j)
                if (rs[i].b < rs[j].e && rs[j].b < rs[i].e) bad = true;
        }
        const size_t z0 = ps.front().off_cell_count;
        const size_t z1 = ps.back().off_cursor + (size_t)ps.back().in.n_frames * kCursorStride * 4;
        for (const Region& r : rs) {
            const bool inside = r.b >= z0 && r.e <= z1;
            const bool outside = r.e <= z0 || r.b >= z1;
            if (r.kind == 0 ? !inside : !outside) bad = true;
        }
        int n_tables = 0;
        for (const Region& r : rs) n_tables += r.kind == 2 && r.b == ps[r.sys].off_thr;
        std::printf("batch layout: %zu systems, %zu regions, %d table copies, cleared block %zu B of %zu %s\n",
                    ps.size(), rs.size(), n_tables, z1 - z0, total, bad ? "FAIL" : "ok");
        if (bad) ++failed;
    }
    return failed;
}
