/* CPU oracle for exact weighted k-means colour quantization.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product path.  Single-threaded, plain
 * C, FP64 distances, exact integer histogram and sums.  Build with
 * -O2 -ffp-contract=off (no FMA contraction, no fast-math).
 *
 * Paper: M. E. Celebi, "Improving the Performance of K-Means for Color
 * Quantization".  Section references below are to that paper.
 *
 * Readings where the paper is silent or loose (each is listed in the design
 * notes of the repository):
 *  - weights are the integer pixel counts n_i; the division by N of Section 2.2
 *    cancels in the weighted mean and in the relative stopping test;
 *  - the first iteration is a full search (Algo. 2 uses m[i] before any
 *    assignment exists); later iterations scan row m[i] of the sorted table;
 *  - each sorted row starts with its own centre and orders the others by
 *    (distance, index); ties in the nearest-centre choice go to the lowest index;
 *  - the pruning test stops only when d[p][t] > 4 prev (1 + 1e-12), so that a
 *    skipped centre is provably farther than c_p despite FP64 rounding;
 *  - an empty cluster keeps its previous centre;
 *  - SSE_i is evaluated after the centre update from exact integer cluster
 *    statistics; stop when (SSE_{i-1} - SSE_i) <= tol * SSE_i, when SSE_i == 0,
 *    or at max_iters;
 *  - random choices use splitmix64 with a fixed draw order (documented below).
 */
#include "cqref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NKEYS (1u << 24)

/* ------------------------------------------------------------------------- */
/* Random numbers: splitmix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast      */
/* splittable pseudorandom number generators", OOPSLA 2014).                 */
/* ------------------------------------------------------------------------- */
uint64_t cqref_splitmix64_next(uint64_t* s)
{
    uint64_t z;
    *s += 0x9E3779B97F4A7C15ull;
    z = *s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Uniform integer in [0, T): draws below (2^64 mod T) are rejected so that the
 * accepted range is a whole number of copies of [0, T). */
uint64_t cqref_uniform_below(uint64_t* s, uint64_t T)
{
    uint64_t reject_below = (0 - T) % T;
    for (;;) {
        uint64_t r = cqref_splitmix64_next(s);
        if (r >= reject_below)
            return r % T;
    }
}

/* ------------------------------------------------------------------------- */
/* Colour helpers                                                            */
/* ------------------------------------------------------------------------- */
static void key_rgb(uint32_t key, int* r, int* g, int* b)
{
    *r = (int)((key >> 16) & 255u);
    *g = (int)((key >> 8) & 255u);
    *b = (int)(key & 255u);
}

/* Squared Euclidean distance between two integer colours (exact). */
static int64_t dist_int(int r0, int g0, int b0, int r1, int g1, int b1)
{
    int64_t dr = r0 - r1, dg = g0 - g1, db = b0 - b1;
    return dr * dr + dg * dg + db * db;
}

/* Squared Euclidean distance, FP64, evaluated as (dx*dx + dy*dy) + dz*dz. */
static double dist_f64(double x0, double x1, double x2, const double* c)
{
    double d0 = x0 - c[0];
    double d1 = x1 - c[1];
    double d2 = x2 - c[2];
    return d0 * d0 + d1 * d1 + d2 * d2;
}

/* ------------------------------------------------------------------------- */
/* Histogram: Section 2.2, items 1 and 2.                                    */
/* The paper finds unique colours with a chained hash table; the result is   */
/* the set of distinct colours with their frequencies, which a dense count    */
/* over all 2^24 colours yields directly, in ascending key order.            */
/* ------------------------------------------------------------------------- */
int cqref_histogram(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride, int32_t subsample,
                    uint32_t* keys, uint32_t* counts, int64_t capacity, int64_t* n_unique)
{
    if (!img || H <= 0 || W <= 0 || row_stride < 3 * (int64_t)W || !n_unique || capacity < 0)
        return CQREF_EINVAL;
    /* Section 2.2 item 1, first method: 2:1 subsampling in both directions
       keeps the pixels at even row and even column */
    const int32_t step = subsample ? 2 : 1;
    if (capacity > 0 && (!keys || !counts))
        return CQREF_EINVAL;
    uint32_t* cnt = (uint32_t*)calloc(NKEYS, sizeof(uint32_t));
    if (!cnt)
        return CQREF_ENOMEM;
    for (int32_t y = 0; y < H; y += step) {
        const uint8_t* row = img + (int64_t)y * row_stride;
        for (int32_t x = 0; x < W; x += step) {
            const uint8_t* p = row + 3 * (int64_t)x;
            uint32_t key = ((uint32_t)p[0] << 16) | ((uint32_t)p[1] << 8) | (uint32_t)p[2];
            cnt[key] += 1u;
        }
    }
    int64_t n = 0;
    for (uint32_t key = 0; key < NKEYS; ++key) {
        if (cnt[key] == 0)
            continue;
        if (n < capacity) {
            keys[n] = key;
            counts[n] = cnt[key];
        }
        ++n;
    }
    free(cnt);
    *n_unique = n;
    return n > capacity ? CQREF_ECAPACITY : CQREF_OK;
}

/* ------------------------------------------------------------------------- */
/* Initialization: Section 2.3.                                              */
/* Draw order (shared definition with any other implementation):            */
/*   FGY: for j = 0..K-1, r_j = j + U(N' - j), swap positions j and r_j of  */
/*        the identity permutation, centre j = colour at position j.         */
/*   MMX: first centre = colour U(N'); then K-1 farthest-first picks (no    */
/*        further draws), ties to the lowest colour index.                   */
/*   KPP: first centre = colour i with the first inclusive prefix of n_i    */
/*        exceeding U(sum n); centre j = colour with the first inclusive     */
/*        prefix of n_i D_i^2 exceeding U(sum n_i D_i^2).                    */
/* U(T) is cqref_uniform_below on one splitmix64 stream seeded with `seed`.  */
/* ------------------------------------------------------------------------- */
static void set_center_from_key(double* c, uint32_t key)
{
    int r, g, b;
    key_rgb(key, &r, &g, &b);
    c[0] = (double)r;
    c[1] = (double)g;
    c[2] = (double)b;
}

/* D_i^2 <- min(D_i^2, |x_i - x_chosen|^2) over all colours. */
static void update_min_d2(const uint32_t* keys, int64_t n, uint32_t chosen_key, int64_t* d2)
{
    int cr, cg, cb;
    key_rgb(chosen_key, &cr, &cg, &cb);
    for (int64_t i = 0; i < n; ++i) {
        int r, g, b;
        key_rgb(keys[i], &r, &g, &b);
        int64_t d = dist_int(r, g, b, cr, cg, cb);
        if (d < d2[i])
            d2[i] = d;
    }
}

/* VAR (Section 2.3, maximum variance), read on the pixel data set: colour i
 * stands for counts[i] identical pixels.  The channel is the one whose pixel
 * variance is largest (compared exactly as N S2 - S1^2; ties to the lower
 * channel, R before G before B).  The N pixels in ascending order of
 * (channel value, key) are cut into K groups [floor(g N / K), floor((g+1) N / K));
 * centre g is the pixel at the group's lower median position. */
static int init_var(const uint32_t* keys, const uint32_t* counts, int64_t n, int32_t K, double* centers)
{
    unsigned __int128 best = 0;
    int ch = 0;
    uint64_t N = 0;
    for (int64_t i = 0; i < n; ++i)
        N += counts[i];
    for (int c = 0; c < 3; ++c) {
        uint64_t s1 = 0;
        unsigned __int128 s2 = 0;
        for (int64_t i = 0; i < n; ++i) {
            const uint64_t x = (keys[i] >> (16 - 8 * c)) & 255u;
            s1 += (uint64_t)counts[i] * x;
            s2 += (unsigned __int128)counts[i] * x * x;
        }
        const unsigned __int128 v = (unsigned __int128)N * s2 - (unsigned __int128)s1 * s1;
        if (c == 0 || v > best) {
            best = v;
            ch = c;
        }
    }
    /* the colours in ascending (channel value, key): a stable counting sort of
       the key-ordered colours by the channel value */
    int64_t* order = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!order)
        return CQREF_ENOMEM;
    int64_t start[257] = {0};
    for (int64_t i = 0; i < n; ++i)
        ++start[((keys[i] >> (16 - 8 * ch)) & 255u) + 1];
    for (int v = 0; v < 256; ++v)
        start[v + 1] += start[v];
    for (int64_t i = 0; i < n; ++i)
        order[start[(keys[i] >> (16 - 8 * ch)) & 255u]++] = i;
    /* walk the pixels in that order */
    int64_t pos = 0;  /* first pixel of order[q] */
    int64_t q = 0;
    for (int32_t g = 0; g < K; ++g) {
        const uint64_t lo = (uint64_t)(((unsigned __int128)g * N) / (unsigned)K);
        const uint64_t hi = (uint64_t)(((unsigned __int128)(g + 1) * N) / (unsigned)K);
        const uint64_t m = lo + (hi - lo - 1) / 2;
        while ((uint64_t)(pos + counts[order[q]]) <= m) {
            pos += counts[order[q]];
            ++q;
        }
        set_center_from_key(centers + 3 * g, keys[order[q]]);
    }
    free(order);
    return CQREF_OK;
}

int64_t cqref_sff_subset(int32_t K, int64_t n)
{
    int64_t L = (int64_t)ceil(2.0 * (double)K * log((double)K));
    if (L < K)
        L = K;
    return L < n ? L : n;
}

/* SFF (Section 2.3, subset farthest first): a uniform subset of L =
 * cqref_sff_subset(K, n) distinct colours, the first L positions of a partial
 * Fisher-Yates shuffle (the draws of FGY), then MMX on the subset in draw
 * order: the first centre is subset[U(L)], then K-1 farthest-first picks by
 * integer D^2 over the subset, ties to the lowest subset position. */
static int init_sff(const uint32_t* keys, int64_t n, int32_t K, uint64_t* rng, double* centers)
{
    const int64_t L = cqref_sff_subset(K, n);
    int64_t* perm = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* d2 = (int64_t*)malloc((size_t)L * sizeof(int64_t));
    if (!perm || !d2) {
        free(perm);
        free(d2);
        return CQREF_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i)
        perm[i] = i;
    for (int64_t j = 0; j < L; ++j) {
        const int64_t r = j + (int64_t)cqref_uniform_below(rng, (uint64_t)(n - j));
        const int64_t t = perm[j];
        perm[j] = perm[r];
        perm[r] = t;
    }
    for (int64_t s = 0; s < L; ++s)
        d2[s] = INT64_MAX;
    int64_t pick = (int64_t)cqref_uniform_below(rng, (uint64_t)L);
    for (int32_t j = 0; j < K; ++j) {
        if (j > 0) {
            int64_t best = -1;
            for (int64_t s = 0; s < L; ++s) {
                if (d2[s] > best) {
                    best = d2[s];
                    pick = s;
                }
            }
        }
        const uint32_t key = keys[perm[pick]];
        set_center_from_key(centers + 3 * j, key);
        int cr, cg, cb;
        key_rgb(key, &cr, &cg, &cb);
        for (int64_t s = 0; s < L; ++s) {
            int r, g, b;
            key_rgb(keys[perm[s]], &r, &g, &b);
            const int64_t d = dist_int(r, g, b, cr, cg, cb);
            if (d < d2[s])
                d2[s] = d;
        }
    }
    free(perm);
    free(d2);
    return CQREF_OK;
}

/* ------------------------------------------------------------------------- */
/* WU as an initializer (Section 3.3, WSM-WU): Wu's greedy orthogonal        */
/* bipartitioning of the colour space (X. Wu, "Efficient statistical         */
/* computations for optimal color quantization", Graphics Gems II, 1991).    */
/* ------------------------------------------------------------------------- */
/* Each channel is cut into 32 levels (value >> 3), giving 32^3 cells.  A box
 * is an inclusive range [lo, hi] of cells per channel.  The statistics of a
 * set of pixels are five exact integers: w (pixels), the channel sums
 * sr, sg, sb, and s2 = the sum of r^2 + g^2 + b^2. */
#define WU_LEVELS 32
#define WU_CELLS (WU_LEVELS * WU_LEVELS * WU_LEVELS)

typedef struct {
    uint64_t m[5]; /* w, sr, sg, sb, s2 */
} wu_mom;

typedef struct {
    int lo[3], hi[3];
} wu_box;

/* |m|^2 / w in FP64, evaluated as ((sr^2 + sg^2) + sb^2) / w. */
static double wu_spread(const wu_mom* a)
{
    const double r = (double)a->m[1], g = (double)a->m[2], b = (double)a->m[3];
    return (r * r + g * g + b * b) / (double)a->m[0];
}

/* Weighted variance (sum of squared deviations from the mean) of a box, in
 * FP64: s2 - |m|^2 / w.  A box of one cell cannot be split and counts 0; a
 * value below zero by rounding also counts 0. */
static double wu_var(const wu_box* b, const wu_mom* tot)
{
    const int vol = (b->hi[0] - b->lo[0] + 1) * (b->hi[1] - b->lo[1] + 1) * (b->hi[2] - b->lo[2] + 1);
    if (vol <= 1 || tot->m[0] == 0)
        return 0.0;
    const double v = (double)tot->m[4] - wu_spread(tot);
    return v > 0.0 ? v : 0.0;
}

/* Statistics of box b summed directly over its cells. */
static void wu_box_moments(const wu_mom* cells, const wu_box* b, wu_mom* out)
{
    memset(out, 0, sizeof *out);
    for (int r = b->lo[0]; r <= b->hi[0]; ++r)
        for (int g = b->lo[1]; g <= b->hi[1]; ++g)
            for (int bl = b->lo[2]; bl <= b->hi[2]; ++bl)
                for (int q = 0; q < 5; ++q)
                    out->m[q] += cells[(r * WU_LEVELS + g) * WU_LEVELS + bl].m[q];
}

/* The best cut of box b: along each channel a, every plane c in
 * [lo_a, hi_a - 1] splits b into [lo_a, c] and [c + 1, hi_a]; a cut leaving
 * either part without pixels is not allowed.  A cut's value is the sum of
 * wu_spread over the two parts (the larger, the smaller their summed squared
 * error); the best cut of a channel is its first one of largest value, and the
 * channel chosen is the one whose best value is largest, ties to R, then G,
 * then B.  Returns 0 if no channel has an allowed cut. */
static int wu_best_cut(const wu_mom* cells, const wu_box* b, const wu_mom* whole, int* axis, int* plane,
                       wu_mom* lower)
{
    double best_v[3] = {0.0, 0.0, 0.0};
    int best_c[3] = {-1, -1, -1};
    wu_mom best_low[3];
    for (int a = 0; a < 3; ++a) {
        /* the box's statistics plane by plane along channel a */
        wu_mom marg[WU_LEVELS];
        memset(marg, 0, sizeof marg);
        for (int r = b->lo[0]; r <= b->hi[0]; ++r)
            for (int g = b->lo[1]; g <= b->hi[1]; ++g)
                for (int bl = b->lo[2]; bl <= b->hi[2]; ++bl) {
                    const int t = a == 0 ? r : a == 1 ? g : bl;
                    for (int q = 0; q < 5; ++q)
                        marg[t].m[q] += cells[(r * WU_LEVELS + g) * WU_LEVELS + bl].m[q];
                }
        wu_mom low;
        memset(&low, 0, sizeof low);
        for (int c = b->lo[a]; c < b->hi[a]; ++c) {
            for (int q = 0; q < 5; ++q)
                low.m[q] += marg[c].m[q];
            wu_mom up;
            for (int q = 0; q < 5; ++q)
                up.m[q] = whole->m[q] - low.m[q];
            if (low.m[0] == 0 || up.m[0] == 0)
                continue;
            const double v = wu_spread(&low) + wu_spread(&up);
            if (v > best_v[a]) {
                best_v[a] = v;
                best_c[a] = c;
                best_low[a] = low;
            }
        }
    }
    int a = 0;
    if (best_v[1] > best_v[a])
        a = 1;
    if (best_v[2] > best_v[a])
        a = 2;
    if (best_c[a] < 0)
        return 0;
    *axis = a;
    *plane = best_c[a];
    *lower = best_low[a];
    return 1;
}

/* Greedy bipartitioning into at most K boxes: starting from the whole grid,
 * repeatedly split the box of largest wu_var (ties to the lowest box index)
 * at its best cut; the lower part keeps the box's index and the upper part
 * becomes the next box.  A box without an allowed cut gets variance 0 and is
 * never chosen again; the process ends at K boxes or when every variance is
 * 0.  Returns the number of boxes. */
static int wu_partition(const wu_mom* cells, int32_t K, wu_box* boxes, wu_mom* mom)
{
    double var[256];
    for (int a = 0; a < 3; ++a) {
        boxes[0].lo[a] = 0;
        boxes[0].hi[a] = WU_LEVELS - 1;
    }
    wu_box_moments(cells, &boxes[0], &mom[0]);
    var[0] = wu_var(&boxes[0], &mom[0]);
    int nb = 1;
    while (nb < K) {
        int next = 0;
        for (int k = 1; k < nb; ++k)
            if (var[k] > var[next])
                next = k;
        if (var[next] <= 0.0)
            break;
        int axis, plane;
        wu_mom low;
        if (!wu_best_cut(cells, &boxes[next], &mom[next], &axis, &plane, &low)) {
            var[next] = 0.0;
            continue;
        }
        boxes[nb] = boxes[next];
        boxes[next].hi[axis] = plane;
        boxes[nb].lo[axis] = plane + 1;
        for (int q = 0; q < 5; ++q)
            mom[nb].m[q] = mom[next].m[q] - low.m[q];
        mom[next] = low;
        var[next] = wu_var(&boxes[next], &mom[next]);
        var[nb] = wu_var(&boxes[nb], &mom[nb]);
        ++nb;
    }
    return nb;
}

static int wu_cells(const uint32_t* keys, const uint32_t* counts, int64_t n, wu_mom** out)
{
    wu_mom* cells = (wu_mom*)calloc(WU_CELLS, sizeof(wu_mom));
    if (!cells)
        return CQREF_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        int r, g, b;
        key_rgb(keys[i], &r, &g, &b);
        wu_mom* c = &cells[((r >> 3) * WU_LEVELS + (g >> 3)) * WU_LEVELS + (b >> 3)];
        const uint64_t w = counts[i];
        c->m[0] += w;
        c->m[1] += w * (uint64_t)r;
        c->m[2] += w * (uint64_t)g;
        c->m[3] += w * (uint64_t)b;
        c->m[4] += w * (uint64_t)(r * r + g * g + b * b);
    }
    *out = cells;
    return CQREF_OK;
}

/* WU initialization: the boxes' weighted means (FP64 quotients of the exact
 * sums).  If the partition ends with fewer than K boxes, the remaining
 * centres repeat the first box's mean (a repeated centre loses every tie to
 * the lower index, so its cluster stays empty). */
static int init_wu(const uint32_t* keys, const uint32_t* counts, int64_t n, int32_t K, double* centers)
{
    wu_mom* cells;
    int rc = wu_cells(keys, counts, n, &cells);
    if (rc)
        return rc;
    wu_box boxes[256];
    wu_mom mom[256];
    const int nb = wu_partition(cells, K, boxes, mom);
    for (int32_t k = 0; k < K; ++k) {
        const wu_mom* m = &mom[k < nb ? k : 0];
        for (int c = 0; c < 3; ++c)
            centers[3 * k + c] = (double)m->m[1 + c] / (double)m->m[0];
    }
    free(cells);
    return CQREF_OK;
}

/* LBG (Section 2.3, splitting; Linde, Buzo and Gray 1980).  The first centre
 * is the weighted mean of the colours (FP64 quotients of the exact sums).  A
 * stage doubles the m centres: centre j becomes c_j - eps, kept at index j,
 * and c_j + eps, appended at index m + j, with eps = (1, 1, 1); when K is not
 * a power of two the last stage splits only the first K - m centres.  After
 * every stage the centres are refined by weighted Lloyd iterations (Algo. 1
 * with the weights of Section 2.2) stopped by the rule of Section 3.3 with the
 * paper's threshold 0.001, at most 100 iterations. */
#define LBG_EPS 1.0
#define LBG_TOL 0.001
#define LBG_MAX_ITERS 100

static int init_lbg(const uint32_t* keys, const uint32_t* counts, int64_t n, int32_t K, double* centers)
{
    uint64_t N = 0, S[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        int r, g, b;
        key_rgb(keys[i], &r, &g, &b);
        N += counts[i];
        S[0] += (uint64_t)counts[i] * (uint64_t)r;
        S[1] += (uint64_t)counts[i] * (uint64_t)g;
        S[2] += (uint64_t)counts[i] * (uint64_t)b;
    }
    for (int c = 0; c < 3; ++c)
        centers[c] = (double)S[c] / (double)N;
    uint8_t* assign = (uint8_t*)malloc((size_t)n);
    if (!assign)
        return CQREF_ENOMEM;
    int32_t m = 1;
    int rc = CQREF_OK;
    while (m < K && rc == CQREF_OK) {
        const int32_t split = 2 * m <= K ? m : K - m;
        for (int32_t j = 0; j < split; ++j)
            for (int c = 0; c < 3; ++c) {
                const double v = centers[3 * j + c];
                centers[3 * (m + j) + c] = v + LBG_EPS;
                centers[3 * j + c] = v - LBG_EPS;
            }
        m += split;
        rc = cqref_kmeans(keys, counts, n, m, centers, LBG_MAX_ITERS, LBG_TOL, 0, assign, NULL, NULL, NULL);
    }
    free(assign);
    return rc;
}

/* DEN (Section 2.3, density-based; Al-Daoud and Roberts 1996).  The colour
 * cube is cut uniformly into M = 8^3 cells (value >> 5 per channel, cell
 * index (r >> 5) * 64 + (g >> 5) * 8 + (b >> 5)).  Cell c holding u_c of the
 * n unique colours gets floor(K u_c / n) centres, and the K - (sum of those)
 * centres left go one each to the cells of largest remainder (K u_c mod n),
 * ties to the lower cell index; a quota never exceeds u_c.  Then, cell by cell
 * in index order, the quota is drawn uniformly without replacement from the
 * cell's colours in key order, as FGY draws (a partial Fisher-Yates shuffle,
 * draw j uniform in [j, u_c)), all from the one splitmix64 stream; the centres
 * follow in that order. */
#define DEN_CELLS 512

static int den_cell(uint32_t key)
{
    return (int)(((key >> 21) & 7u) * 64u + ((key >> 13) & 7u) * 8u + ((key >> 5) & 7u));
}

int cqref_den_quotas(const uint32_t* keys, int64_t n, int32_t K, int32_t* quota)
{
    if (!keys || !quota || n < 1 || K < 1 || K > 256 || K > n)
        return CQREF_EINVAL;
    int64_t u[DEN_CELLS] = {0};
    for (int64_t i = 0; i < n; ++i)
        ++u[den_cell(keys[i])];
    int64_t rem[DEN_CELLS];
    int32_t given = 0;
    for (int c = 0; c < DEN_CELLS; ++c) {
        quota[c] = (int32_t)(((int64_t)K * u[c]) / n);
        rem[c] = ((int64_t)K * u[c]) % n;
        given += quota[c];
    }
    for (int32_t left = K - given; left > 0; --left) {
        int best = -1;
        for (int c = 0; c < DEN_CELLS; ++c)
            if (rem[c] > 0 && (best < 0 || rem[c] > rem[best]))
                best = c;
        ++quota[best];
        rem[best] = 0;
    }
    return CQREF_OK;
}

static int init_den(const uint32_t* keys, int64_t n, int32_t K, uint64_t* rng, double* centers)
{
    int32_t quota[DEN_CELLS];
    int rc = cqref_den_quotas(keys, n, K, quota);
    if (rc)
        return rc;
    /* the colours of each cell in key order */
    int64_t start[DEN_CELLS + 1] = {0};
    for (int64_t i = 0; i < n; ++i)
        ++start[den_cell(keys[i]) + 1];
    for (int c = 0; c < DEN_CELLS; ++c)
        start[c + 1] += start[c];
    int64_t* order = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!order)
        return CQREF_ENOMEM;
    int64_t fill[DEN_CELLS];
    memcpy(fill, start, sizeof fill);
    for (int64_t i = 0; i < n; ++i)
        order[fill[den_cell(keys[i])]++] = i;
    int32_t k = 0;
    for (int c = 0; c < DEN_CELLS; ++c) {
        int64_t* cell = order + start[c];
        const int64_t uc = start[c + 1] - start[c];
        for (int32_t j = 0; j < quota[c]; ++j) {
            const int64_t r = j + (int64_t)cqref_uniform_below(rng, (uint64_t)(uc - j));
            const int64_t t = cell[j];
            cell[j] = cell[r];
            cell[r] = t;
            set_center_from_key(centers + 3 * k, keys[cell[j]]);
            ++k;
        }
    }
    free(order);
    return CQREF_OK;
}

int cqref_wu_boxes(const uint32_t* keys, const uint32_t* counts, int64_t n, int32_t K, int32_t* boxes,
                   int32_t* n_boxes)
{
    if (!keys || !counts || !boxes || !n_boxes || n < 1 || K < 1 || K > 256)
        return CQREF_EINVAL;
    wu_mom* cells;
    int rc = wu_cells(keys, counts, n, &cells);
    if (rc)
        return rc;
    wu_box bx[256];
    wu_mom mom[256];
    const int nb = wu_partition(cells, K, bx, mom);
    for (int k = 0; k < nb; ++k)
        for (int a = 0; a < 3; ++a) {
            boxes[6 * k + a] = bx[k].lo[a];
            boxes[6 * k + 3 + a] = bx[k].hi[a];
        }
    *n_boxes = nb;
    free(cells);
    return CQREF_OK;
}

int cqref_init(const uint32_t* keys, const uint32_t* counts, int64_t n, int32_t K,
               int32_t scheme, uint64_t seed, double* centers, int32_t* k_used)
{
    if (!keys || !counts || !centers || n < 1 || K < 1 || K > 256)
        return CQREF_EINVAL;
    if (scheme < CQREF_INIT_FORGY || scheme > CQREF_INIT_DEN)
        return CQREF_EINVAL;
    if (n <= K) {
        /* Fewer colours than palette entries: every colour is a centre. */
        for (int32_t k = 0; k < K; ++k) {
            if (k < n)
                set_center_from_key(centers + 3 * k, keys[k]);
            else
                centers[3 * k] = centers[3 * k + 1] = centers[3 * k + 2] = 0.0;
        }
        if (k_used)
            *k_used = (int32_t)n;
        return CQREF_OK;
    }
    if (k_used)
        *k_used = K;
    if (scheme == CQREF_INIT_USER)
        return CQREF_OK;

    uint64_t rng = seed;
    if (scheme == CQREF_INIT_VAR)
        return init_var(keys, counts, n, K, centers);
    if (scheme == CQREF_INIT_SFF)
        return init_sff(keys, n, K, &rng, centers);
    if (scheme == CQREF_INIT_WU)
        return init_wu(keys, counts, n, K, centers);
    if (scheme == CQREF_INIT_LBG)
        return init_lbg(keys, counts, n, K, centers);
    if (scheme == CQREF_INIT_DEN)
        return init_den(keys, n, K, &rng, centers);
    if (scheme == CQREF_INIT_FORGY) {
        int64_t* perm = (int64_t*)malloc((size_t)n * sizeof(int64_t));
        if (!perm)
            return CQREF_ENOMEM;
        for (int64_t i = 0; i < n; ++i)
            perm[i] = i;
        for (int32_t j = 0; j < K; ++j) {
            int64_t r = j + (int64_t)cqref_uniform_below(&rng, (uint64_t)(n - j));
            int64_t t = perm[j];
            perm[j] = perm[r];
            perm[r] = t;
            set_center_from_key(centers + 3 * j, keys[perm[j]]);
        }
        free(perm);
        return CQREF_OK;
    }

    int64_t* d2 = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!d2)
        return CQREF_ENOMEM;
    for (int64_t i = 0; i < n; ++i)
        d2[i] = INT64_MAX;

    int64_t first;
    if (scheme == CQREF_INIT_MAXMIN) {
        first = (int64_t)cqref_uniform_below(&rng, (uint64_t)n);
    } else {
        uint64_t total = 0;
        for (int64_t i = 0; i < n; ++i)
            total += counts[i];
        uint64_t r = cqref_uniform_below(&rng, total);
        uint64_t prefix = 0;
        first = n - 1;
        for (int64_t i = 0; i < n; ++i) {
            prefix += counts[i];
            if (prefix > r) {
                first = i;
                break;
            }
        }
    }
    set_center_from_key(centers, keys[first]);
    update_min_d2(keys, n, keys[first], d2);

    for (int32_t j = 1; j < K; ++j) {
        int64_t pick = -1;
        if (scheme == CQREF_INIT_MAXMIN) {
            int64_t best = -1;
            for (int64_t i = 0; i < n; ++i) {
                if (d2[i] > best) {
                    best = d2[i];
                    pick = i;
                }
            }
        } else {
            uint64_t total = 0;
            for (int64_t i = 0; i < n; ++i)
                total += (uint64_t)counts[i] * (uint64_t)d2[i];
            uint64_t r = cqref_uniform_below(&rng, total);
            uint64_t prefix = 0;
            for (int64_t i = 0; i < n; ++i) {
                prefix += (uint64_t)counts[i] * (uint64_t)d2[i];
                if (prefix > r) {
                    pick = i;
                    break;
                }
            }
        }
        set_center_from_key(centers + 3 * j, keys[pick]);
        update_min_d2(keys, n, keys[pick], d2);
    }
    free(d2);
    return CQREF_OK;
}

/* ------------------------------------------------------------------------- */
/* Weighted Lloyd / Weighted Sort-Means: Algo. 1, Algo. 2, Section 3.3.      */
/* ------------------------------------------------------------------------- */

/* Exact unsigned 128-bit value converted to double by the fixed rule
 * hi * 2^64 + lo, each conversion and the sum rounded to nearest. */
static double u128_to_f64(unsigned __int128 v)
{
    uint64_t hi = (uint64_t)(v >> 64);
    uint64_t lo = (uint64_t)v;
    return (double)hi * 18446744073709551616.0 + (double)lo;
}

int cqref_kmeans(const uint32_t* keys, const uint32_t* counts, int64_t n, int32_t K,
                 double* centers, int32_t max_iters, double tol, int32_t prune,
                 uint8_t* assign, uint8_t* palette, double* sse_trace, cqref_stats* stats)
{
    if (!keys || !counts || !centers || !assign || n < 1 || K < 1 || K > 256 || max_iters < 1)
        return CQREF_EINVAL;
    if (!(tol >= 0.0))
        return CQREF_EINVAL;

    cqref_stats st;
    memset(&st, 0, sizeof st);
    st.prune = prune ? 1 : 0;
    st.n_unique = n;
    uint64_t n_pixels = 0;
    for (int64_t i = 0; i < n; ++i)
        n_pixels += counts[i];

    if (n <= K) {
        /* Exact optimum: one centre per colour, SSE 0, no iteration needed. */
        for (int32_t k = 0; k < K; ++k) {
            if (k < n)
                set_center_from_key(centers + 3 * k, keys[k]);
            else
                centers[3 * k] = centers[3 * k + 1] = centers[3 * k + 2] = 0.0;
        }
        for (int64_t i = 0; i < n; ++i)
            assign[i] = (uint8_t)i;
        st.k_used = (int32_t)n;
        st.converged = 1;
    } else {
        st.k_used = K;
        double* D = (double*)malloc(sizeof(double) * (size_t)K * (size_t)K);
        int32_t* M = (int32_t*)malloc(sizeof(int32_t) * (size_t)K * (size_t)K);
        uint64_t* cn = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)K);
        uint64_t* cs = (uint64_t*)malloc(sizeof(uint64_t) * 3 * (size_t)K);
        uint64_t* cq = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)K);
        if (!D || !M || !cn || !cs || !cq) {
            free(D); free(M); free(cn); free(cs); free(cq);
            return CQREF_ENOMEM;
        }
        double sse_prev = 0.0;
        for (int32_t it = 1; it <= max_iters; ++it) {
            const int pruned_pass = prune && it >= 2;
            if (pruned_pass) {
                /* Pairwise centre distances and, per row a, the permutation of
                 * centres by increasing distance from c_a (a itself first). */
                for (int32_t a = 0; a < K; ++a)
                    for (int32_t b = 0; b < K; ++b)
                        D[a * K + b] = dist_f64(centers[3 * a], centers[3 * a + 1],
                                                centers[3 * a + 2], centers + 3 * b);
                for (int32_t a = 0; a < K; ++a) {
                    int32_t* row = M + a * K;
                    int32_t len = 0;
                    row[len++] = a;
                    for (int32_t b = 0; b < K; ++b) {
                        if (b == a)
                            continue;
                        /* insertion by (distance, index) */
                        int32_t pos = len;
                        while (pos > 1) {
                            int32_t o = row[pos - 1];
                            double dox = D[a * K + o], dbx = D[a * K + b];
                            if (dox > dbx || (dox == dbx && o > b)) {
                                row[pos] = o;
                                --pos;
                            } else {
                                break;
                            }
                        }
                        row[pos] = b;
                        ++len;
                    }
                }
            }

            /* Assignment step. */
            for (int64_t i = 0; i < n; ++i) {
                int r, g, b;
                key_rgb(keys[i], &r, &g, &b);
                const double x0 = (double)r, x1 = (double)g, x2 = (double)b;
                int32_t best;
                double bd, second = -1.0;
                int have_second = 0;
                int64_t evals;
                if (!pruned_pass) {
                    best = 0;
                    bd = dist_f64(x0, x1, x2, centers);
                    for (int32_t k = 1; k < K; ++k) {
                        double d = dist_f64(x0, x1, x2, centers + 3 * k);
                        if (d < bd) {
                            second = bd;
                            bd = d;
                            best = k;
                        } else if (!have_second || d < second) {
                            second = d;
                        }
                        have_second = 1;
                    }
                    evals = K;
                } else {
                    const int32_t p = assign[i];
                    const double prev = dist_f64(x0, x1, x2, centers + 3 * p);
                    const double limit = 4.0 * prev * (1.0 + 1e-12);
                    best = p;
                    bd = prev;
                    evals = 1;
                    for (int32_t j = 1; j < K; ++j) {
                        const int32_t t = M[p * K + j];
                        if (D[p * K + t] > limit)
                            break;
                        double d = dist_f64(x0, x1, x2, centers + 3 * t);
                        ++evals;
                        if (d < bd || (d == bd && t < best)) {
                            second = bd;
                            bd = d;
                            best = t;
                        } else if (!have_second || d < second) {
                            second = d;
                        }
                        have_second = 1;
                    }
                }
                if (have_second && (second - bd) <= 1e-5 * second)
                    st.near_ties += 1;
                st.ndc_total += evals;
                assign[i] = (uint8_t)best;
            }

            /* Update step: exact integer cluster statistics. */
            memset(cn, 0, sizeof(uint64_t) * (size_t)K);
            memset(cs, 0, sizeof(uint64_t) * 3 * (size_t)K);
            memset(cq, 0, sizeof(uint64_t) * (size_t)K);
            for (int64_t i = 0; i < n; ++i) {
                int r, g, b;
                key_rgb(keys[i], &r, &g, &b);
                const uint64_t w = counts[i];
                const int32_t k = assign[i];
                cn[k] += w;
                cs[3 * k + 0] += w * (uint64_t)r;
                cs[3 * k + 1] += w * (uint64_t)g;
                cs[3 * k + 2] += w * (uint64_t)b;
                cq[k] += w * (uint64_t)(r * r + g * g + b * b);
            }
            /* Weighted means (the last line of Algo. 2); empty clusters stay. */
            for (int32_t k = 0; k < K; ++k) {
                if (cn[k] == 0)
                    continue;
                centers[3 * k + 0] = (double)cs[3 * k + 0] / (double)cn[k];
                centers[3 * k + 1] = (double)cs[3 * k + 1] / (double)cn[k];
                centers[3 * k + 2] = (double)cs[3 * k + 2] / (double)cn[k];
            }
            /* SSE of eq. (1) with the exact means:
             * sum_k (n_k Q_k - |S_k|^2) / n_k, numerator in exact 128-bit. */
            double sse = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                if (cn[k] == 0)
                    continue;
                unsigned __int128 nq = (unsigned __int128)cn[k] * cq[k];
                unsigned __int128 s2 = (unsigned __int128)cs[3 * k] * cs[3 * k]
                                     + (unsigned __int128)cs[3 * k + 1] * cs[3 * k + 1]
                                     + (unsigned __int128)cs[3 * k + 2] * cs[3 * k + 2];
                sse += u128_to_f64(nq - s2) / (double)cn[k];
            }
            if (sse_trace)
                sse_trace[it - 1] = sse;
            st.iters = it;
            st.sse_final = sse;
            /* Stopping rule of Section 3.3 (Linde et al.), multiplied through. */
            if (sse == 0.0 || (it >= 2 && (sse_prev - sse) <= tol * sse)) {
                st.converged = 1;
                break;
            }
            sse_prev = sse;
        }
        free(D); free(M); free(cn); free(cs); free(cq);
    }
    st.mse_float = st.sse_final / (double)n_pixels;
    if (palette) {
        for (int32_t k = 0; k < K; ++k) {
            for (int c = 0; c < 3; ++c) {
                /* round half up, clamped to [0, 255]: floor(c + 0.5) */
                const double v = centers[3 * k + c] + 0.5;
                int q;
                if (!(v >= 1.0))
                    q = 0;
                else if (v >= 256.0)
                    q = 255;
                else
                    q = (int)v; /* v >= 1: truncation is floor */
                palette[3 * k + c] = (uint8_t)q;
            }
        }
    }
    if (stats)
        *stats = st;
    return CQREF_OK;
}

/* ------------------------------------------------------------------------- */
/* Pixel mapping and MSE: Section 1 (mapping phase), Section 3.1 (MSE).      */
/* Each pixel goes to the palette entry at the smallest integer squared      */
/* distance, lowest index on ties.  The answer depends only on the colour,   */
/* so it is memoised per colour.                                             */
/* ------------------------------------------------------------------------- */
int cqref_map(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride,
              const uint8_t* palette, int32_t K, uint8_t* out_idx, uint8_t* out_rgb,
              uint64_t* sq_err_sum)
{
    if (!img || !palette || H <= 0 || W <= 0 || row_stride < 3 * (int64_t)W || K < 1 || K > 256)
        return CQREF_EINVAL;
    int16_t* memo = (int16_t*)malloc(sizeof(int16_t) * (size_t)NKEYS);
    if (!memo)
        return CQREF_ENOMEM;
    memset(memo, 0xff, sizeof(int16_t) * (size_t)NKEYS); /* -1: not yet known */
    uint64_t err = 0;
    for (int32_t y = 0; y < H; ++y) {
        const uint8_t* row = img + (int64_t)y * row_stride;
        for (int32_t x = 0; x < W; ++x) {
            const uint8_t* p = row + 3 * (int64_t)x;
            uint32_t key = ((uint32_t)p[0] << 16) | ((uint32_t)p[1] << 8) | (uint32_t)p[2];
            int32_t idx = memo[key];
            if (idx < 0) {
                int64_t bd = INT64_MAX;
                for (int32_t k = 0; k < K; ++k) {
                    int64_t d = dist_int(p[0], p[1], p[2], palette[3 * k], palette[3 * k + 1],
                                         palette[3 * k + 2]);
                    if (d < bd) {
                        bd = d;
                        idx = k;
                    }
                }
                memo[key] = (int16_t)idx;
            }
            const uint8_t* q = palette + 3 * idx;
            err += (uint64_t)dist_int(p[0], p[1], p[2], q[0], q[1], q[2]);
            const int64_t o = (int64_t)y * W + x;
            if (out_idx)
                out_idx[o] = (uint8_t)idx;
            if (out_rgb) {
                out_rgb[3 * o + 0] = q[0];
                out_rgb[3 * o + 1] = q[1];
                out_rgb[3 * o + 2] = q[2];
            }
        }
    }
    free(memo);
    if (sq_err_sum)
        *sq_err_sum = err;
    return CQREF_OK;
}

int cqref_quantize(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride, int32_t subsample,
                   int32_t K, int32_t scheme, uint64_t seed, int32_t max_iters, double tol, int32_t prune,
                   uint8_t* palette, uint8_t* out_idx, uint8_t* out_rgb, cqref_stats* stats)
{
    if (!img || !palette || H <= 0 || W <= 0 || K < 1 || K > 256 || scheme == CQREF_INIT_USER)
        return CQREF_EINVAL;
    int64_t cap = (int64_t)H * W, n = 0;
    uint32_t* keys = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)cap);
    uint32_t* counts = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)cap);
    uint8_t* assign = (uint8_t*)malloc((size_t)cap);
    double centers[256 * 3];
    int rc = CQREF_ENOMEM;
    if (!keys || !counts || !assign)
        goto out;
    rc = cqref_histogram(img, H, W, row_stride, subsample, keys, counts, cap, &n);
    if (rc)
        goto out;
    rc = cqref_init(keys, counts, n, K, scheme, seed, centers, NULL);
    if (rc)
        goto out;
    cqref_stats st;
    rc = cqref_kmeans(keys, counts, n, K, centers, max_iters, tol, prune, assign, palette, NULL, &st);
    if (rc)
        goto out;
    uint64_t err = 0;
    rc = cqref_map(img, H, W, row_stride, palette, st.k_used, out_idx, out_rgb, &err);
    if (rc)
        goto out;
    st.mse_img = (double)err / ((double)H * (double)W);
    if (stats)
        *stats = st;
out:
    free(keys);
    free(counts);
    free(assign);
    return rc;
}
