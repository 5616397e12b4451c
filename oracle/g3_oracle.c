/*
 * g3 oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU statement of what the triplet correlation histogram
 * g3(r12, r13, r23) of Sec. 3.3 (Eq. 3 and the triplet conditions that follow
 * it; the serial logic of the "Serial logic for triplet correlation function"
 * listing) computes.  It exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can check the HIP library against it; no
 * product code may link or call it, and it shares no code with the library.
 *
 * What it computes (readings of the paper recorded in the design notes):
 *   * positions are integers in an orthorhombic periodic box L = (Lx, Ly, Lz),
 *     0 <= x_d < L_d; rmax is an exact binary64 value in the same unit;
 *   * bins: thr[b] = ceil((b * rmax / nbins)^2), b = 0..nbins, in exact
 *     rational arithmetic; an integer squared distance s lies in bin
 *     b(s) = max{b : thr[b] <= s} if s < thr[nbins] (= R2) and is cut otherwise
 *     (half-open bins of width rmax/nbins, strict cutoff r < rmax);
 *   * minimum image per component: d = x_j - x_i; d -= L if 2d > L,
 *     d += L if 2d < -L (rmax < L_d / 2 makes the tie irrelevant);
 *   * for every frame, centre i and ORDERED pair (j, k) of distinct atoms,
 *     both different from i: d_ij = mi(x_j - x_i), d_ik = mi(x_k - x_i), and
 *     the third side is taken from the "updated positions" the serial listing
 *     stores, d_jk = d_ik - d_ij, WITHOUT a second minimum image.  If all three
 *     squared lengths are below R2, H_full[b_ij][b_ik][b_jk] += 1;
 *   * the half layout counts unordered pairs: H_half[lo][hi][c] with
 *     lo <= hi is H_full[lo][hi][c] off the diagonal and H_full[a][a][c] / 2 on
 *     it (folded here from H_full so that symmetry is tested, not assumed);
 *   * the pair histogram H2[b] counts ordered pairs (i, j), j != i, with
 *     b_ij = b (the g2 histogram computed beside g3).
 *
 * Integers are int64 throughout (no overflow concerns, no pre-tests).  The
 * only parallelism is an OpenMP split of centres with private histograms
 * that are summed at the end (integer sums, so the result is exact).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

#define G3O_MAX_NBINS 512

/* Exact thresholds thr[b] = ceil((b * rmax / nbins)^2) for b = 0..count
 * (bins of width rmax / nbins; count >= nbins extends them past rmax).
 * rmax is decomposed as m * 2^e with m odd (or e >= 0), which makes the
 * square an exact rational b^2 m^2 2^(2e) / nbins^2.  Returns 0, or -1 for
 * arguments outside 1 <= rmax < 2^31, 1 <= nbins <= count <= 512. */
int g3o_thresholds_n(double rmax, int nbins, int count, uint64_t *thr)
{
    if (!(rmax >= 1.0) || !(rmax < 2147483648.0) || nbins < 1 || count < nbins ||
        count > G3O_MAX_NBINS)
        return -1;
    int E;
    double f = frexp(rmax, &E);                 /* rmax = f * 2^E, f in [0.5, 1) */
    int64_t m = (int64_t)ldexp(f, 53);          /* exact 53-bit integer */
    int e = E - 53;
    while ((m & 1) == 0 && e < 0) { m >>= 1; e++; }
    for (int b = 0; b <= count; b++) {
        u128 q;
        u128 den = (u128)nbins * (u128)nbins;
        if (e >= 0) {
            u128 R = ((u128)b * (u128)m) << e;  /* b * rmax, exact integer */
            u128 num = R * R;
            q = (num + den - 1) / den;
        } else {
            u128 num = (u128)b * (u128)b * (u128)m * (u128)m;
            den <<= (2 * (-e));
            q = (num + den - 1) / den;
        }
        thr[b] = (uint64_t)q;
    }
    return 0;
}

int g3o_thresholds(double rmax, int nbins, uint64_t *thr)
{
    return g3o_thresholds_n(rmax, nbins, nbins, thr);
}

/* b(s) = max{b : thr[b] <= s}; -1 if s >= thr[nbins]. */
int g3o_bin(uint64_t s, const uint64_t *thr, int nbins)
{
    if (s >= thr[nbins]) return -1;
    int b = nbins - 1;
    while (thr[b] > s) b--;
    return b;
}

static int64_t mi(int64_t d, int64_t L)
{
    if (2 * d > L) d -= L;
    else if (2 * d < -L) d += L;
    return d;
}

static int check_args(const int32_t *box, double rmax, int nbins, int n_atoms)
{
    if (n_atoms < 0 || nbins < 1 || nbins > G3O_MAX_NBINS) return -1;
    for (int d = 0; d < 3; d++)
        if (box[d] <= 0 || !(2.0 * rmax < (double)box[d])) return -1;
    return 0;
}

typedef struct { int64_t d[3]; int b; } nbr_t;

/* Neighbours of centre i in one frame: every j != i with |mi(x_j - x_i)|^2 < R2,
 * in index order.  Returns the count. */
static int neighbours(const int32_t *fr, int N, const int32_t *box, int i,
                      const uint64_t *thr, int nbins, nbr_t *out)
{
    const int32_t *X = fr, *Y = fr + N, *Z = fr + 2 * (size_t)N;
    int n = 0;
    for (int j = 0; j < N; j++) {
        if (j == i) continue;
        int64_t dx = mi((int64_t)X[j] - X[i], box[0]);
        int64_t dy = mi((int64_t)Y[j] - Y[i], box[1]);
        int64_t dz = mi((int64_t)Z[j] - Z[i], box[2]);
        uint64_t s = (uint64_t)(dx * dx + dy * dy + dz * dz);
        int b = g3o_bin(s, thr, nbins);
        if (b < 0) continue;
        out[n].d[0] = dx; out[n].d[1] = dy; out[n].d[2] = dz; out[n].b = b;
        n++;
    }
    return n;
}

/* H_full ([b_ij][b_ik][b_jk], nbins x nbins x nbins_third, row-major) over
 * all frames.  The two sides at the centre are below rmax (nbins bins of
 * width rmax / nbins); the third side, from the updated positions, is binned
 * in nbins_third bins of the same width, i.e. kept below
 * nbins_third * rmax / nbins.  nbins_third = nbins is the one-cutoff reading;
 * nbins_third = 2 nbins with rmax = L/4 is the paper's geometry (two sides
 * below L/4, the third below L/2, Sec. 3.3).
 * frames: [n_frames][3][n_atoms] int32.  Adds into H (caller zeroes it).
 * n_threads <= 0 uses the OpenMP default.  If centres != NULL only the
 * listed centre indices (n_centres of them) contribute.  Returns 0 or -1. */
int g3o_hist_full3(const int32_t *frames, int n_frames, int n_atoms, const int32_t *box,
                   double rmax, int nbins, int nbins_third, uint64_t *H, int n_threads,
                   const int32_t *centres, int n_centres)
{
    if (check_args(box, rmax, nbins, n_atoms)) return -1;
    if (nbins_third < nbins || nbins_third > 2 * nbins) return -1;
    uint64_t thr[G3O_MAX_NBINS + 1];
    if (g3o_thresholds_n(rmax, nbins, nbins_third, thr)) return -1;
    const int nc = nbins_third;
    const size_t nb3 = (size_t)nbins * nbins * nc;
    const int n_ctr = centres ? n_centres : n_atoms;
    int nt = 1;
#ifdef _OPENMP
    nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#endif
    uint64_t *priv = calloc((size_t)nt * nb3, sizeof(uint64_t));
    if (!priv) return -1;
    int err = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        uint64_t *Ht = priv + (size_t)t * nb3;
        nbr_t *nb = malloc(sizeof(nbr_t) * (size_t)(n_atoms > 0 ? n_atoms : 1));
        if (!nb) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            err = 1;
        }
        for (int f = 0; f < n_frames && nb; f++) {
            const int32_t *fr = frames + (size_t)f * 3 * n_atoms;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
            for (int ci = 0; ci < n_ctr; ci++) {
                int i = centres ? centres[ci] : ci;
                int n = neighbours(fr, n_atoms, box, i, thr, nbins, nb);
                for (int p = 0; p < n; p++) {
                    for (int q = 0; q < n; q++) {
                        if (q == p) continue;
                        int64_t ex = nb[q].d[0] - nb[p].d[0];
                        int64_t ey = nb[q].d[1] - nb[p].d[1];
                        int64_t ez = nb[q].d[2] - nb[p].d[2];
                        int c = g3o_bin((uint64_t)(ex * ex + ey * ey + ez * ez), thr, nc);
                        if (c < 0) continue;
                        Ht[((size_t)nb[p].b * nbins + nb[q].b) * nc + c] += 1;
                    }
                }
            }
        }
        free(nb);
    }
    if (!err)
        for (int t = 0; t < nt; t++)
            for (size_t x = 0; x < nb3; x++) H[x] += priv[(size_t)t * nb3 + x];
    free(priv);
    return err ? -1 : 0;
}

int g3o_hist_full(const int32_t *frames, int n_frames, int n_atoms, const int32_t *box,
                  double rmax, int nbins, uint64_t *H, int n_threads,
                  const int32_t *centres, int n_centres)
{
    return g3o_hist_full3(frames, n_frames, n_atoms, box, rmax, nbins, nbins, H, n_threads,
                          centres, n_centres);
}

/* Pair histogram of ORDERED pairs (i, j), i != j, |mi(x_j - x_i)| < rmax,
 * binned like the triplet sides.  Adds into H2[nbins].  Centres are split
 * over n_threads OpenMP threads (<= 0: the default) with private counts. */
int g3o_pair_hist(const int32_t *frames, int n_frames, int n_atoms, const int32_t *box,
                  double rmax, int nbins, uint64_t *H2, int n_threads)
{
    if (check_args(box, rmax, nbins, n_atoms)) return -1;
    uint64_t thr[G3O_MAX_NBINS + 1];
    if (g3o_thresholds(rmax, nbins, thr)) return -1;
    int nt = 1;
#ifdef _OPENMP
    nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#endif
    uint64_t *priv = calloc((size_t)nt * nbins, sizeof(uint64_t));
    if (!priv) return -1;
    int err = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        uint64_t *Ht = priv + (size_t)t * nbins;
        nbr_t *nb = malloc(sizeof(nbr_t) * (size_t)(n_atoms > 0 ? n_atoms : 1));
        if (!nb) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            err = 1;
        }
        for (int f = 0; f < n_frames && nb; f++) {
            const int32_t *fr = frames + (size_t)f * 3 * n_atoms;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
            for (int i = 0; i < n_atoms; i++) {
                int n = neighbours(fr, n_atoms, box, i, thr, nbins, nb);
                for (int p = 0; p < n; p++) Ht[nb[p].b] += 1;
            }
        }
        free(nb);
    }
    if (!err)
        for (int t = 0; t < nt; t++)
            for (int b = 0; b < nbins; b++) H2[b] += priv[(size_t)t * nbins + b];
    free(priv);
    return err ? -1 : 0;
}

/* Half-layout index of (lo, hi, c), lo <= hi: rows lo hold hi = lo..nbins-1. */
/* Half-layout index of (lo, hi, c), lo <= hi: rows lo hold hi = lo..nbins-1,
 * each with nc third-side bins. */
static size_t half_index3(int lo, int hi, int c, int nbins, int nc)
{
    size_t rowoff = (size_t)lo * nbins - (size_t)lo * (lo - 1) / 2;
    return (rowoff + (size_t)(hi - lo)) * nc + c;
}


size_t g3o_half_len3(int nbins, int nc)
{
    return (size_t)nbins * (nbins + 1) / 2 * nc;
}

size_t g3o_half_len(int nbins)
{
    return g3o_half_len3(nbins, nbins);
}

/* Fold H_full (nbins x nbins x nc) into the half layout.  Returns the number
 * of (a, b, c) where the fold is inconsistent (H_full[a][b][c] !=
 * H_full[b][a][c], or an odd diagonal count); 0 means H_full had the
 * symmetry the definition implies. */
long g3o_fold_half3(const uint64_t *full, int nbins, int nc, uint64_t *half)
{
    long bad = 0;
    for (int a = 0; a < nbins; a++)
        for (int b = a; b < nbins; b++)
            for (int c = 0; c < nc; c++) {
                uint64_t v = full[((size_t)a * nbins + b) * nc + c];
                uint64_t w = full[((size_t)b * nbins + a) * nc + c];
                if (a == b) {
                    if (v & 1) bad++;
                    half[half_index3(a, b, c, nbins, nc)] = v / 2;
                } else {
                    if (v != w) bad++;
                    half[half_index3(a, b, c, nbins, nc)] = v;
                }
            }
    return bad;
}

long g3o_fold_half(const uint64_t *full, int nbins, uint64_t *half)
{
    return g3o_fold_half3(full, nbins, nbins, half);
}

/* ---------------------------------------------------------------------------
 * Ideal-gas normalisation (Eq. 3 with U = 0).
 *
 * For i.i.d. uniform positions, the expected number of ordered (j, k) around a
 * centre with |d_ij| in bin a, |d_ik| in bin b and |d_ik - d_ij| in bin c is
 * (N-1)(N-2)/V^2 * W(a, b, c), where W is the 6-D volume
 *     W = 8 pi^2 \int_A \int_B \int_C r s t 1[|r - s| <= t <= r + s] dt ds dr
 * (d^3 r2 = 4 pi r^2 dr, then d^3 r3 = 2 pi s t / r ds dt after substituting
 * t^2 = r^2 + s^2 - 2 r s cos(theta)).  The oracle evaluates it by nested
 * one-dimensional Gauss-Legendre quadrature, splitting each interval at every
 * point where the integrand changes polynomial piece, so every panel is
 * integrated exactly up to rounding.
 * ------------------------------------------------------------------------- */

static const double GL_X[5] = {-0.9061798459386640, -0.5384693101056831, 0.0,
                               0.5384693101056831, 0.9061798459386640};
static const double GL_W[5] = {0.2369268850561891, 0.4786286704993665,
                               0.5688888888888889, 0.4786286704993665,
                               0.2369268850561891};

/* Inner t-integral: \int_{c0}^{c1} t 1[|r-s| <= t <= r+s] dt. */
static double t_integral(double r, double s, double c0, double c1)
{
    double lo = fabs(r - s) > c0 ? fabs(r - s) : c0;
    double hi = (r + s) < c1 ? (r + s) : c1;
    return hi > lo ? 0.5 * (hi * hi - lo * lo) : 0.0;
}

static int cmp_dbl(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Collect the breakpoints of an interval [lo, hi]: the ends plus every
 * candidate in cand[] strictly inside, sorted. */
static int split_points(double lo, double hi, const double *cand, int nc, double *out)
{
    int n = 0;
    out[n++] = lo;
    for (int i = 0; i < nc; i++)
        if (cand[i] > lo && cand[i] < hi) out[n++] = cand[i];
    out[n++] = hi;
    qsort(out, (size_t)n, sizeof(double), cmp_dbl);
    return n;
}

/* \int_{b0}^{b1} s * t_integral(r, s, c0, c1) ds for fixed r.  As a function of
 * s the integrand changes piece where |r - s| or r + s meets c0 or c1. */
static double s_integral(double r, double b0, double b1, double c0, double c1)
{
    double cand[6] = {r - c0, r + c0, r - c1, r + c1, c0 - r, c1 - r};
    double pts[8];
    int np = split_points(b0, b1, cand, 6, pts);
    double acc = 0.0;
    for (int p = 0; p + 1 < np; p++) {
        double m = 0.5 * (pts[p] + pts[p + 1]), h = 0.5 * (pts[p + 1] - pts[p]);
        if (h <= 0) continue;
        for (int g = 0; g < 5; g++) {
            double s = m + h * GL_X[g];
            acc += h * GL_W[g] * s * t_integral(r, s, c0, c1);
        }
    }
    return acc;
}

/* W for the bin box [a0,a1] x [b0,b1] x [c0,c1] (lengths in any unit). */
double g3o_W_box(double a0, double a1, double b0, double b1, double c0, double c1)
{
    /* The s-integral is one polynomial in r as long as the order of the
     * s-breakpoints {r +- c, c - r} and the ends {b0, b1} does not change:
     * a breakpoint meets an end at r = b +- c or c - b, and two breakpoints
     * meet each other at r = c0, c1, (c0 + c1)/2 or (c1 - c0)/2. */
    double cand[16];
    int k = 0;
    double bs[2] = {b0, b1}, cs[2] = {c0, c1};
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            cand[k++] = bs[i] + cs[j];
            cand[k++] = bs[i] - cs[j];
            cand[k++] = cs[j] - bs[i];
        }
    cand[k++] = c0;
    cand[k++] = c1;
    cand[k++] = 0.5 * (c0 + c1);
    cand[k++] = 0.5 * (c1 - c0);
    double pts[20];
    int np = split_points(a0, a1, cand, k, pts);
    double acc = 0.0;
    for (int p = 0; p + 1 < np; p++) {
        double m = 0.5 * (pts[p] + pts[p + 1]), h = 0.5 * (pts[p + 1] - pts[p]);
        if (h <= 0) continue;
        for (int g = 0; g < 5; g++) {
            double r = m + h * GL_X[g];
            acc += h * GL_W[g] * r * s_integral(r, b0, b1, c0, c1);
        }
    }
    return 8.0 * M_PI * M_PI * acc;
}

/* W(a, b, c) for every bin of width dr, full layout [a][b][c], c < nc. */
void g3o_W_table3(int nbins, int nc, double dr, double *W)
{
    for (int a = 0; a < nbins; a++)
        for (int b = 0; b < nbins; b++)
            for (int c = 0; c < nc; c++)
                W[((size_t)a * nbins + b) * nc + c] =
                    g3o_W_box(a * dr, (a + 1) * dr, b * dr, (b + 1) * dr, c * dr, (c + 1) * dr);
}

void g3o_W_table(int nbins, double dr, double *W)
{
    g3o_W_table3(nbins, nbins, dr, W);
}

/* g3 = H / E with E = F N (N-1)(N-2) / V^2 * W (ordered pairs, full layout);
 * in the half layout E is halved on the diagonal lo == hi.  g3 = 0 where W = 0.
 * H and g3 have the layout's length; W is the full table from g3o_W_table. */
void g3o_normalize3(const uint64_t *H, int layout_full, int nbins, int nc, const double *W,
                    int64_t n_frames, int64_t n_atoms, const int32_t *box, double *g3)
{
    double V = (double)box[0] * (double)box[1] * (double)box[2];
    double Nd = (double)n_atoms;
    double pref = (double)n_frames * Nd * (Nd - 1.0) * (Nd - 2.0) / (V * V);
    if (layout_full) {
        size_t n = (size_t)nbins * nbins * nc;
        for (size_t x = 0; x < n; x++) {
            double E = pref * W[x];
            g3[x] = E > 0 ? (double)H[x] / E : 0.0;
        }
    } else {
        for (int a = 0; a < nbins; a++)
            for (int b = a; b < nbins; b++)
                for (int c = 0; c < nc; c++) {
                    double E = pref * W[((size_t)a * nbins + b) * nc + c];
                    if (a == b) E *= 0.5;
                    size_t x = half_index3(a, b, c, nbins, nc);
                    g3[x] = E > 0 ? (double)H[x] / E : 0.0;
                }
    }
}

void g3o_normalize(const uint64_t *H, int layout_full, int nbins, const double *W,
                   int64_t n_frames, int64_t n_atoms, const int32_t *box, double *g3)
{
    g3o_normalize3(H, layout_full, nbins, nbins, W, n_frames, n_atoms, box, g3);
}

/* g2(r) from the ordered pair histogram (the paper computes g2 beside g3,
 * Sec. 3.3): an ideal gas puts N(N-1)/V ordered pairs per unit volume, so
 * shell b, between r_b = b*dr and r_{b+1}, expects
 * F * N(N-1)/V * (4 pi / 3)(r_{b+1}^3 - r_b^3). */
void g3o_normalize_pairs(const uint64_t *H2, int nbins, double rmax, int64_t n_frames,
                         int64_t n_atoms, const int32_t *box, double *g2)
{
    double V = (double)box[0] * (double)box[1] * (double)box[2];
    double Nd = (double)n_atoms;
    double dr = rmax / nbins;
    for (int b = 0; b < nbins; b++) {
        double r0 = dr * b, r1 = dr * (b + 1);
        double shell = 4.0 * M_PI / 3.0 * (r1 * r1 * r1 - r0 * r0 * r0);
        double E = (double)n_frames * Nd * (Nd - 1.0) / V * shell;
        g2[b] = E > 0 ? (double)H2[b] / E : 0.0;
    }
}

int g3o_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
