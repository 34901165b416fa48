/*
 * Seeded synthetic CSR generators (structure only, int32 indices).
 *
 * These produce the input matrices for the tests, the benchmark and the
 * serving driver.  They stand in for the SuiteSparse matrices the paper
 * evaluates on (Table II), which are not redistributed here: the shapes,
 * row-length distributions and sparsity patterns follow the workloads named
 * in the benchmark configurations (uniform, R-MAT, banded, block-diagonal,
 * Zipf row lengths, 27-point stencil).
 *
 * Nothing in this file computes any part of the prediction method (no
 * intermediate-product counts, no sampling, no distinct counting).  Random
 * numbers come from a counter-based stream built on the MurmurHash3 64-bit
 * finaliser (Appleby), keyed by (seed, generator id, shape, row) so every row
 * is generated independently and the result does not depend on the thread
 * count.  The prediction's own row sampler uses a different generator.
 *
 * Two-phase protocol for the row-wise generators: *_rowlen() fills the length
 * of every row, the caller turns that into a row-pointer array, then *_fill()
 * writes the column indices of every row, sorted ascending and distinct.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- random */

static inline uint64_t fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

/* ctr-th random word of the stream named by key */
static inline uint64_t wl_word(uint64_t key, uint64_t ctr)
{
    return fmix64(key ^ fmix64(ctr * 0xd1342543de82ef95ULL + 0x632be59bd9b4e019ULL));
}

/* uniform integer in [0, w) (multiply-shift; bias below 2^-32 for w < 2^32) */
static inline uint64_t wl_below(uint64_t r, uint64_t w)
{
    return (uint64_t)(((unsigned __int128)r * (unsigned __int128)w) >> 64);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double wl_unit(uint64_t r)
{
    return (double)(r >> 11) * (1.0 / 9007199254740992.0);
}

static inline uint64_t wl_row_key(uint64_t base, int64_t row)
{
    return fmix64(base ^ fmix64((uint64_t)row + 0x9fb21c651e98df25ULL));
}

/* base key of one matrix: generator id, shape and seed */
uint64_t wl_matrix_key(uint64_t seed, uint32_t gen_id, int64_t nrows, int64_t ncols, int64_t d)
{
    uint64_t k = fmix64(seed + 0x2545f4914f6cdd1dULL);
    k = fmix64(k ^ ((uint64_t)gen_id * 0x9e6c63d0676a9a99ULL));
    k = fmix64(k ^ (uint64_t)nrows);
    k = fmix64(k ^ ((uint64_t)ncols << 1));
    k = fmix64(k ^ ((uint64_t)d * 0xa0761d6478bd642fULL));
    return k;
}

/* ------------------------------------------------- distinct column draws */

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

static void sort_i32(int32_t* v, int64_t n)
{
    if (n <= 32) {
        for (int64_t i = 1; i < n; ++i) {
            int32_t x = v[i];
            int64_t j = i - 1;
            while (j >= 0 && v[j] > x) { v[j + 1] = v[j]; --j; }
            v[j + 1] = x;
        }
    } else {
        qsort(v, (size_t)n, sizeof(int32_t), cmp_i32);
    }
}

/*
 * Write L distinct values drawn uniformly from [lo, lo + w) into out, sorted.
 * The draws consume the stream (key, ctr0, ctr0+1, ...).  Needs L <= w.
 * For L > w/2 the complement (w - L excluded values) is drawn instead.
 */
static void draw_distinct(uint64_t key, uint64_t ctr0, int64_t lo, int64_t w, int64_t L,
                          int32_t* out)
{
    if (L <= 0) return;
    if (L == w) {
        for (int64_t j = 0; j < L; ++j) out[j] = (int32_t)(lo + j);
        return;
    }
    int complement = (L > w / 2);
    int64_t want = complement ? (w - L) : L;
    /* open-addressing set of the drawn offsets; size a power of two >= 2*want */
    int64_t cap = 16;
    while (cap < 2 * want) cap <<= 1;
    int64_t* set = (int64_t*)malloc((size_t)cap * sizeof(int64_t));
    for (int64_t j = 0; j < cap; ++j) set[j] = -1;
    int64_t got = 0;
    uint64_t ctr = ctr0;
    int32_t* drawn = complement ? (int32_t*)malloc((size_t)(want > 0 ? want : 1) * sizeof(int32_t)) : out;
    while (got < want) {
        int64_t x = (int64_t)wl_below(wl_word(key, ctr++), (uint64_t)w);
        uint64_t h = ((uint64_t)x * 0x9e3779b97f4a7c15ULL) >> 11;
        int64_t s = (int64_t)(h & (uint64_t)(cap - 1));
        while (set[s] != -1 && set[s] != x) s = (s + 1) & (cap - 1);
        if (set[s] == -1) {
            set[s] = x;
            drawn[got++] = (int32_t)x;
        }
    }
    if (!complement) {
        for (int64_t j = 0; j < L; ++j) out[j] += (int32_t)lo;
        sort_i32(out, L);
    } else {
        sort_i32(drawn, want);
        int64_t a = 0, o = 0;
        for (int64_t x = 0; x < w; ++x) {
            if (a < want && drawn[a] == x) { ++a; continue; }
            out[o++] = (int32_t)(lo + x);
        }
        free(drawn);
    }
    free(set);
}

/* ----------------------------------------------------- row-wise families */

enum {
    WL_UNIFORM = 1,   /* d distinct uniform columns in [0, ncols)                 */
    WL_BANDED = 2,    /* d distinct uniform columns in [i - p, i + p] (p = param) */
    WL_BLOCKDIAG = 3, /* d distinct uniform columns in the block of row i (param) */
    WL_ZIPF = 4,      /* Zipf(param/1000) row length, uniform distinct columns    */
};

typedef struct {
    int kind;
    int64_t nrows, ncols, d, param;
    uint64_t key;
    const double* zipf_cdf; /* WL_ZIPF: cdf[x-1] = P(X <= x), x in [1, ncols] */
    double zipf_mean;       /* WL_ZIPF: E[X] */
} wl_rowgen;

static void row_window(const wl_rowgen* g, int64_t i, int64_t* lo, int64_t* w)
{
    switch (g->kind) {
    case WL_BANDED: {
        int64_t a = i - g->param, b = i + g->param + 1;
        if (a < 0) a = 0;
        if (b > g->ncols) b = g->ncols;
        if (b < a) b = a;
        *lo = a; *w = b - a;
        return;
    }
    case WL_BLOCKDIAG: {
        int64_t a = (i / g->param) * g->param, b = a + g->param;
        if (a > g->ncols) a = g->ncols;
        if (b > g->ncols) b = g->ncols;
        *lo = a; *w = b - a;
        return;
    }
    default:
        *lo = 0; *w = g->ncols;
        return;
    }
}

static int64_t row_length(const wl_rowgen* g, int64_t i)
{
    int64_t lo, w;
    row_window(g, i, &lo, &w);
    int64_t L = g->d;
    if (g->kind == WL_ZIPF) {
        uint64_t key = wl_row_key(g->key, i);
        double u = wl_unit(wl_word(key, 0));
        /* smallest x with cdf(x) > u */
        int64_t a = 0, b = g->ncols - 1;
        while (a < b) {
            int64_t m = (a + b) / 2;
            if (g->zipf_cdf[m] > u) b = m; else a = m + 1;
        }
        double x = (double)(a + 1);
        double len = floor((double)g->d * x / g->zipf_mean + 0.5);
        L = (int64_t)len;
        if (L < 1) L = 1;
    }
    if (L > w) L = w;
    if (L < 0) L = 0;
    return L;
}

static int setup(wl_rowgen* g, int kind, int64_t nrows, int64_t ncols, int64_t d, int64_t param,
                 uint64_t seed, double** cdf_out)
{
    memset(g, 0, sizeof(*g));
    g->kind = kind;
    g->nrows = nrows;
    g->ncols = ncols;
    g->d = d;
    g->param = param;
    g->key = wl_matrix_key(seed, (uint32_t)kind, nrows, ncols, d * 1000003 + param);
    *cdf_out = NULL;
    if (kind == WL_BLOCKDIAG && param <= 0) return -1;
    if (kind == WL_ZIPF) {
        if (ncols <= 0) return -1;
        double s = (double)param / 1000.0;
        double* cdf = (double*)malloc((size_t)ncols * sizeof(double));
        if (!cdf) return -2;
        double z = 0.0, m = 0.0;
        for (int64_t x = 1; x <= ncols; ++x) {
            double p = pow((double)x, -s);
            z += p;
            m += p * (double)x;
            cdf[x - 1] = z;
        }
        for (int64_t x = 0; x < ncols; ++x) cdf[x] /= z;
        cdf[ncols - 1] = 2.0; /* every u < 1 lands inside the table */
        g->zipf_cdf = cdf;
        g->zipf_mean = m / z;
        *cdf_out = cdf;
    }
    return 0;
}

int wl_rowgen_rowlen(int kind, int64_t nrows, int64_t ncols, int64_t d, int64_t param,
                     uint64_t seed, int32_t* rowlen, double* realised_mean)
{
    wl_rowgen g;
    double* cdf;
    int rc = setup(&g, kind, nrows, ncols, d, param, seed, &cdf);
    if (rc) return rc;
    int64_t total = 0;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int64_t i = 0; i < nrows; ++i) {
        int64_t L = row_length(&g, i);
        rowlen[i] = (int32_t)L;
        total += L;
    }
    if (realised_mean) *realised_mean = nrows ? (double)total / (double)nrows : 0.0;
    free(cdf);
    return 0;
}

int wl_rowgen_fill(int kind, int64_t nrows, int64_t ncols, int64_t d, int64_t param,
                   uint64_t seed, const int64_t* rpt, int32_t* col)
{
    wl_rowgen g;
    double* cdf;
    int rc = setup(&g, kind, nrows, ncols, d, param, seed, &cdf);
    if (rc) return rc;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < nrows; ++i) {
        int64_t lo, w;
        row_window(&g, i, &lo, &w);
        int64_t L = rpt[i + 1] - rpt[i];
        draw_distinct(wl_row_key(g.key, i), 1, lo, w, L, col + rpt[i]);
    }
    free(cdf);
    return 0;
}

/* ------------------------------------------------- 27-point 3-D stencil */

/* row (z*n + y)*n + x couples to every grid neighbour (x+dx, y+dy, z+dz),
 * dx, dy, dz in {-1, 0, 1}, that lies inside the n^3 grid; natural order */
int wl_stencil27_rowlen(int64_t n, int32_t* rowlen)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n * n * n; ++r) {
        int64_t x = r % n, y = (r / n) % n, z = r / (n * n);
        int64_t cx = 1 + (x > 0) + (x < n - 1);
        int64_t cy = 1 + (y > 0) + (y < n - 1);
        int64_t cz = 1 + (z > 0) + (z < n - 1);
        rowlen[r] = (int32_t)(cx * cy * cz);
    }
    return 0;
}

int wl_stencil27_fill(int64_t n, const int64_t* rpt, int32_t* col)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n * n * n; ++r) {
        int64_t x = r % n, y = (r / n) % n, z = r / (n * n);
        int64_t o = rpt[r];
        for (int64_t dz = -1; dz <= 1; ++dz)
            for (int64_t dy = -1; dy <= 1; ++dy)
                for (int64_t dx = -1; dx <= 1; ++dx) {
                    int64_t X = x + dx, Y = y + dy, Z = z + dz;
                    if (X < 0 || Y < 0 || Z < 0 || X >= n || Y >= n || Z >= n) continue;
                    col[o++] = (int32_t)((Z * n + Y) * n + X);
                }
    }
    return 0;
}

/* ---------------------------------------------------------------- R-MAT */

/*
 * Plain R-MAT (Chakrabarti, Zhan & Faloutsos, SDM 2004): each of nedges edges
 * descends `scale` levels, choosing quadrant (0,0), (0,1), (1,0), (1,1) with
 * probabilities a, b, c, 1-a-b-c.  No noise and no vertex permutation.  An
 * edge that lands outside [0,nrows) x [0,ncols) (only possible when nrows or
 * ncols is not 2^scale) is redrawn from the next attempt of its own stream.
 * Duplicates are merged; rows come out sorted.
 *
 * Output arrays are malloc'ed here and released with wl_free().
 */
int wl_rmat(int scale, int64_t nrows, int64_t ncols, int64_t nedges, double a, double b, double c,
            uint64_t seed, int64_t** rpt_out, int32_t** col_out, int64_t* nnz_out)
{
    if (scale < 0 || scale > 31 || nrows <= 0 || ncols <= 0 || nedges < 0) return -1;
    if (nrows > ((int64_t)1 << scale) || ncols > ((int64_t)1 << scale)) return -1;
    uint64_t key = wl_matrix_key(seed, 5u, nrows, ncols, nedges);
    double ab = a + b, abc = a + b + c;
    int32_t* er = (int32_t*)malloc((size_t)(nedges ? nedges : 1) * sizeof(int32_t));
    int32_t* ec = (int32_t*)malloc((size_t)(nedges ? nedges : 1) * sizeof(int32_t));
    int64_t* cnt = (int64_t*)calloc((size_t)nrows + 1, sizeof(int64_t));
    if (!er || !ec || !cnt) { free(er); free(ec); free(cnt); return -2; }

#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nedges; ++e) {
        uint64_t ekey = wl_row_key(key, e);
        uint64_t ctr = 0;
        for (;;) {
            int64_t r = 0, cc = 0;
            for (int l = 0; l < scale; ++l) {
                double u = wl_unit(wl_word(ekey, ctr++));
                int rb, cb;
                if (u < a) { rb = 0; cb = 0; }
                else if (u < ab) { rb = 0; cb = 1; }
                else if (u < abc) { rb = 1; cb = 0; }
                else { rb = 1; cb = 1; }
                r = (r << 1) | rb;
                cc = (cc << 1) | cb;
            }
            if (r < nrows && cc < ncols) { er[e] = (int32_t)r; ec[e] = (int32_t)cc; break; }
        }
    }
    /* bucket the edges by row (counting sort), then sort + merge each row */
    for (int64_t e = 0; e < nedges; ++e) cnt[er[e] + 1]++;
    for (int64_t i = 0; i < nrows; ++i) cnt[i + 1] += cnt[i];
    int32_t* bucket = (int32_t*)malloc((size_t)(nedges ? nedges : 1) * sizeof(int32_t));
    int64_t* pos = (int64_t*)malloc((size_t)nrows * sizeof(int64_t));
    if (!bucket || !pos) { free(er); free(ec); free(cnt); free(bucket); free(pos); return -2; }
    memcpy(pos, cnt, (size_t)nrows * sizeof(int64_t));
    for (int64_t e = 0; e < nedges; ++e) bucket[pos[er[e]]++] = ec[e];
    free(er);
    free(ec);
    int64_t* uniq = pos; /* reuse: distinct count per row */
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < nrows; ++i) {
        int32_t* v = bucket + cnt[i];
        int64_t n = cnt[i + 1] - cnt[i];
        sort_i32(v, n);
        int64_t u = 0;
        for (int64_t j = 0; j < n; ++j)
            if (u == 0 || v[u - 1] != v[j]) v[u++] = v[j];
        uniq[i] = u;
    }
    int64_t* rpt = (int64_t*)malloc((size_t)(nrows + 1) * sizeof(int64_t));
    rpt[0] = 0;
    for (int64_t i = 0; i < nrows; ++i) rpt[i + 1] = rpt[i] + uniq[i];
    int32_t* col = (int32_t*)malloc((size_t)(rpt[nrows] ? rpt[nrows] : 1) * sizeof(int32_t));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nrows; ++i)
        memcpy(col + rpt[i], bucket + cnt[i], (size_t)uniq[i] * sizeof(int32_t));
    free(bucket);
    free(pos);
    free(cnt);
    *rpt_out = rpt;
    *col_out = col;
    *nnz_out = rpt[nrows];
    return 0;
}

void wl_free(void* p) { free(p); }

int wl_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
