/*
 * Serial CPU oracle for sampled-compression-ratio structure prediction
 * (Du et al., "Predicting the Output Structure of Sparse Matrix Multiplication
 * with Sampled Compression Ratio", arXiv 2207.13848).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * statement of what the GPU library computes.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load it.  It shares no source,
 * header, table or helper with the HIP path, and the product never calls it.
 *
 * Everything here is serial and plain: loops, qsort, unsigned __int128.
 *
 * Conventions (all readings are listed with their reasons in the design notes):
 *  - A is M x K, B is K x N, both CSR with int32 row pointers and column
 *    indices (Sec. II-A, II-B).  Only the structure is used; there are no
 *    values.  Rows may be unsorted and may hold duplicate entries: the
 *    intermediate-product count counts stored entries, the distinct count
 *    counts distinct columns.
 *  - Loop ranges over row pointers are half-open, [rpt[i], rpt[i+1]).
 *  - Counts are unsigned 64-bit; products that can exceed 64 bits use
 *    unsigned __int128.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* Mirror of the library's statistics block, declared here independently. */
typedef struct {
    uint64_t total_flop;  /* F: intermediate products of the whole product           */
    uint64_t n_sampled;   /* n_s: number of sampled rows (draws, for the paper mode) */
    uint64_t sample_flop; /* f*: intermediate products of the sampled rows           */
    uint64_t sample_nnz;  /* z*: distinct output columns of the sampled rows         */
    uint64_t out_sum;     /* sum of the per-row output                               */
    uint64_t nrows;       /* M                                                       */
    uint64_t flags;       /* bit 0: empty sample (fallback)                          */
    uint64_t a_sample_nnz; /* stored entries of A in the sampled rows (per draw)     */
} orc_stats;

#define ORC_FLAG_EMPTY_SAMPLE 1u

enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_DIM = -2, ORC_ERR_CSR = -8, ORC_ERR_MEM = -5 };

/* ------------------------------------------------------------ validation */

/* rpt[0] = 0, non-decreasing, rpt[nrows] = nnz; every column in [0, ncols). */
int orc_check_csr(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t* rpt, const int32_t* col)
{
    if (nrows < 0 || ncols < 0 || nnz < 0) return ORC_ERR_ARG;
    if (rpt[0] != 0 || (int64_t)rpt[nrows] != nnz) return ORC_ERR_CSR;
    for (int64_t i = 0; i < nrows; ++i)
        if (rpt[i + 1] < rpt[i]) return ORC_ERR_CSR;
    for (int64_t j = 0; j < nnz; ++j)
        if (col[j] < 0 || (int64_t)col[j] >= ncols) return ORC_ERR_CSR;
    return ORC_OK;
}

/* ------------------------------------------- Sec. V-A, Alg. 1: row FLOP */

/*
 * Intermediate products of output row i under the row-wise dataflow, Eq. (1):
 * every stored A(i,k) meets every stored entry of B row k, so the count is
 * the sum over A's row i of the length of the B row its column names.
 */
uint64_t orc_row_flop_one(int64_t i, const int32_t* Arpt, const int32_t* Acol, const int32_t* Brpt)
{
    uint64_t f = 0;
    for (int64_t j = Arpt[i]; j < Arpt[i + 1]; ++j) {
        int32_t k = Acol[j];
        f += (uint64_t)(Brpt[k + 1] - Brpt[k]);
    }
    return f;
}

/* Alg. 1: the count of every row and their total F = FLOP(C). */
void orc_row_flop(int64_t M, const int32_t* Arpt, const int32_t* Acol, const int32_t* Brpt,
                  uint64_t* row_flop, uint64_t* total)
{
    uint64_t F = 0;
    for (int64_t i = 0; i < M; ++i) {
        uint64_t f = orc_row_flop_one(i, Arpt, Acol, Brpt);
        if (row_flop) row_flop[i] = f;
        F += f;
    }
    *total = F;
}

/* ----------------------------------------- Sec. IV-B: exact row NNZ of C */

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/*
 * Exact number of distinct columns of output row i: gather the columns of
 * every B row that A's row i names (the intermediate products, Eq. (1)),
 * sort them and count the distinct values.  The paper counts with a hash
 * table (Alg. 2); any exact method gives the same number.
 * buf must hold orc_row_flop_one(i) entries.
 */
uint64_t orc_row_nnz_one(int64_t i, const int32_t* Arpt, const int32_t* Acol, const int32_t* Brpt,
                         const int32_t* Bcol, int32_t* buf)
{
    int64_t n = 0;
    for (int64_t j = Arpt[i]; j < Arpt[i + 1]; ++j) {
        int32_t k = Acol[j];
        for (int64_t q = Brpt[k]; q < Brpt[k + 1]; ++q) buf[n++] = Bcol[q];
    }
    if (n == 0) return 0;
    qsort(buf, (size_t)n, sizeof(int32_t), cmp_i32);
    uint64_t distinct = 1;
    for (int64_t q = 1; q < n; ++q)
        if (buf[q] != buf[q - 1]) ++distinct;
    return distinct;
}

/* ----------------------------------------------- row sampling (Sec. IV-A) */

/*
 * splitmix64 (Steele, Lea & Flood, OOPSLA 2014; Vigna's public-domain
 * splitmix64.c): the generator state advances by the golden-ratio increment
 * 0x9E3779B97F4A7C15 and each output is the state passed through the
 * finaliser below.  orc_splitmix64(seed, i) is the (i+1)-th output of the
 * stream whose initial state is seed.
 */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1u) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* 53-bit acceptance threshold of a per-row sampling probability `rate`. */
uint64_t orc_rate_threshold(double rate)
{
    if (!(rate > 0.0)) return 0;                   /* also rejects NaN */
    if (rate >= 1.0) return (uint64_t)1 << 53;
    return (uint64_t)(rate * 9007199254740992.0);  /* floor; exact in binary64 */
}

/*
 * Row sample of A (Sec. IV-A: rows of A only; B is reached through them).
 * Bernoulli mode: row i is sampled iff the top 53 bits of
 * orc_splitmix64(seed, i) fall below T.  Rows come out ascending.
 */
int64_t orc_sample_bernoulli(int64_t M, uint64_t seed, uint64_t T, int32_t* rows)
{
    int64_t n = 0;
    for (int64_t i = 0; i < M; ++i)
        if ((orc_splitmix64(seed, (uint64_t)i) >> 11) < T) rows[n++] = (int32_t)i;
    return n;
}

/*
 * The paper's own sampler (Alg. 2 and the sample-size rule of Sec. V-B):
 * sample_num = min(floor(0.003 M), 300) draws; draw r picks row
 * floor(M * u_r) with u_r a uniform number in [0, 1), with replacement.  The
 * uniform numbers are u_r = (splitmix64(seed, r) >> 11) * 2^-53, so
 * floor(M * u_r) = (M * (splitmix64(seed, r) >> 11)) >> 53 exactly.
 */
int64_t orc_paper_sample_num(int64_t M)
{
    int64_t s = (int64_t)(0.003 * (double)M); /* floor for M >= 0 */
    return s < 300 ? s : 300;
}

int64_t orc_sample_paper(int64_t M, uint64_t seed, int32_t* rows)
{
    int64_t n = orc_paper_sample_num(M);
    for (int64_t r = 0; r < n; ++r) {
        uint64_t u53 = orc_splitmix64(seed, (uint64_t)r) >> 11;
        rows[r] = (int32_t)(((u128)(uint64_t)M * u53) >> 53);
    }
    return n;
}

/* ----------------------------------------------------------- helpers */

static uint64_t ceil_div_u128(u128 num, u128 den) { return (uint64_t)((num + den - 1) / den); }

/*
 * ceil(a * q / d) for a 64-bit a and 128-bit q and d (0 < d < 2^127) whose
 * quotient is below 2^64: binary long division of the 192-bit product.  Its
 * top 128 bits (bits 64..191) are then below d, so they are the first partial
 * remainder, and the 64 low bits are brought down one at a time, each giving
 * one quotient bit.  Returns UINT64_MAX when the quotient does not fit (which
 * the reference design never asks for).
 */
uint64_t orc_ceil_mul_div_wide(uint64_t a, uint64_t q_hi, uint64_t q_lo, uint64_t d_hi,
                               uint64_t d_lo)
{
    u128 d = ((u128)d_hi << 64) | d_lo;
    u128 low = (u128)a * q_lo;                    /* a times the low half of q  */
    u128 high = (u128)a * q_hi;                   /* a times the high half of q */
    uint64_t bits_lo = (uint64_t)low;             /* bits 0..63 of a q          */
    u128 rem = (low >> 64) + high;                /* bits 64..191 of a q        */
    if (d == 0 || (d >> 127) != 0 || rem >= d) return UINT64_MAX;
    uint64_t quo = 0;
    for (int b = 63; b >= 0; --b) {
        rem = (rem << 1) | ((bits_lo >> b) & 1u);
        quo <<= 1;
        if (rem >= d) {
            rem -= d;
            quo |= 1u;
        }
    }
    return quo + (rem != 0);
}

/*
 * The sampled part of Alg. 2: f* (sample_flop) and z* (sample_nnz) summed
 * over the sampled rows (duplicates count once per draw), and n_s.
 */
static int sample_sums(int64_t M, const int32_t* Arpt, const int32_t* Acol, const int32_t* Brpt,
                       const int32_t* Bcol, double rate, uint64_t seed, int paper_mode,
                       orc_stats* st)
{
    int32_t* rows = (int32_t*)malloc((size_t)(M > 0 ? M : 1) * sizeof(int32_t));
    if (!rows) return ORC_ERR_MEM;
    int64_t n = paper_mode ? orc_sample_paper(M, seed, rows)
                           : orc_sample_bernoulli(M, seed, orc_rate_threshold(rate), rows);
    uint64_t maxf = 0;
    for (int64_t s = 0; s < n; ++s) {
        uint64_t f = orc_row_flop_one(rows[s], Arpt, Acol, Brpt);
        if (f > maxf) maxf = f;
    }
    int32_t* buf = (int32_t*)malloc((size_t)(maxf > 0 ? maxf : 1) * sizeof(int32_t));
    if (!buf) { free(rows); return ORC_ERR_MEM; }
    uint64_t fs = 0, zs = 0, as = 0;
    for (int64_t s = 0; s < n; ++s) {
        fs += orc_row_flop_one(rows[s], Arpt, Acol, Brpt);
        zs += orc_row_nnz_one(rows[s], Arpt, Acol, Brpt, Bcol, buf);
        as += (uint64_t)(Arpt[rows[s] + 1] - Arpt[rows[s]]);
    }
    free(buf);
    free(rows);
    st->n_sampled = (uint64_t)n;
    st->sample_flop = fs;
    st->sample_nnz = zs;
    st->a_sample_nnz = as;
    return ORC_OK;
}

/* -------------------- the proposed method: Sec. IV-D, Eq. (4), Alg. 2 */

/*
 * Predicted structure of C = A.B.  The sampled compression ratio is
 * r* = f* / z* and each row is predicted as its FLOP divided by r*, i.e.
 * nnz_pred[i] = ceil(row_flop[i] * z* / f*), computed exactly.  The predicted
 * total is Z2* = F z* / f*, kept as the integers (F, z*, f*).
 * If f* = 0 the ratio is undefined; every row then falls back to its FLOP
 * (the upper bound) and the empty-sample flag is set.
 */
int orc_predict(int64_t M, int64_t K, const int32_t* Arpt, const int32_t* Acol,
                const int32_t* Brpt, const int32_t* Bcol, double rate, uint64_t seed,
                int paper_mode, int64_t* nnz_pred, uint64_t* row_flop_out, orc_stats* st)
{
    (void)K;
    if (M < 0 || !(rate >= 0.0 && rate <= 1.0)) return ORC_ERR_ARG;
    memset(st, 0, sizeof(*st));
    st->nrows = (uint64_t)M;
    uint64_t* rf = (uint64_t*)malloc((size_t)(M > 0 ? M : 1) * sizeof(uint64_t));
    if (!rf) return ORC_ERR_MEM;
    orc_row_flop(M, Arpt, Acol, Brpt, rf, &st->total_flop);
    int rc = sample_sums(M, Arpt, Acol, Brpt, Bcol, rate, seed, paper_mode, st);
    if (rc) { free(rf); return rc; }
    uint64_t sum = 0;
    if (st->sample_flop == 0) {
        st->flags |= ORC_FLAG_EMPTY_SAMPLE;
        for (int64_t i = 0; i < M; ++i) { nnz_pred[i] = (int64_t)rf[i]; sum += rf[i]; }
    } else {
        for (int64_t i = 0; i < M; ++i) {
            uint64_t p = ceil_div_u128((u128)rf[i] * st->sample_nnz, st->sample_flop);
            nnz_pred[i] = (int64_t)p;
            sum += p;
        }
    }
    st->out_sum = sum;
    if (row_flop_out) memcpy(row_flop_out, rf, (size_t)M * sizeof(uint64_t));
    free(rf);
    return ORC_OK;
}

/* ----------------------- the reference design: Sec. IV-C, Eq. (2) */

/*
 * The existing estimator on the same sample: Z1* = z* / p with p the realised
 * sampled proportion n_s / M, so Z1* = z* M / n_s.  The compression ratio is
 * F / Z1* and each row is predicted as ceil(row_flop[i] * Z1* / F)
 * = ceil(row_flop[i] * z* * M / (n_s * F)).  Not clamped.  Fallback as in
 * orc_predict when f* = 0.  Every value fits: z* <= n_s N (no sampled row has
 * more than N columns) and row_flop[i] <= F, so the quotient is at most
 * M N < 2^62; the numerator, though, can reach 2^155 (row_flop < 2^62,
 * z* M < 2^93), so it is divided as a 192-bit number.
 */
int orc_reference(int64_t M, int64_t K, const int32_t* Arpt, const int32_t* Acol,
                  const int32_t* Brpt, const int32_t* Bcol, double rate, uint64_t seed,
                  int paper_mode, int64_t* nnz_ref, orc_stats* st)
{
    (void)K;
    if (M < 0 || !(rate >= 0.0 && rate <= 1.0)) return ORC_ERR_ARG;
    memset(st, 0, sizeof(*st));
    st->nrows = (uint64_t)M;
    uint64_t* rf = (uint64_t*)malloc((size_t)(M > 0 ? M : 1) * sizeof(uint64_t));
    if (!rf) return ORC_ERR_MEM;
    orc_row_flop(M, Arpt, Acol, Brpt, rf, &st->total_flop);
    int rc = sample_sums(M, Arpt, Acol, Brpt, Bcol, rate, seed, paper_mode, st);
    if (rc) { free(rf); return rc; }
    uint64_t sum = 0;
    if (st->sample_flop == 0) {
        st->flags |= ORC_FLAG_EMPTY_SAMPLE;
        for (int64_t i = 0; i < M; ++i) { nnz_ref[i] = (int64_t)rf[i]; sum += rf[i]; }
    } else {
        u128 q = (u128)st->sample_nnz * (uint64_t)M;  /* z* M  (< 2^93) */
        u128 d = (u128)st->n_sampled * st->total_flop; /* n_s F (< 2^93) */
        for (int64_t i = 0; i < M; ++i) {
            uint64_t v = orc_ceil_mul_div_wide(rf[i], (uint64_t)(q >> 64), (uint64_t)q,
                                               (uint64_t)(d >> 64), (uint64_t)d);
            nnz_ref[i] = (int64_t)v;
            sum += v;
        }
    }
    st->out_sum = sum;
    free(rf);
    return ORC_OK;
}

/* ------------------------------- the precise method (Sec. I, symbolic) */

/* Exact nnz of every output row; out_sum = Z = NNZ(C). */
int orc_exact(int64_t M, int64_t K, const int32_t* Arpt, const int32_t* Acol, const int32_t* Brpt,
              const int32_t* Bcol, int64_t* nnz_exact, orc_stats* st)
{
    (void)K;
    if (M < 0) return ORC_ERR_ARG;
    memset(st, 0, sizeof(*st));
    st->nrows = (uint64_t)M;
    uint64_t maxf = 0, F = 0;
    for (int64_t i = 0; i < M; ++i) {
        uint64_t f = orc_row_flop_one(i, Arpt, Acol, Brpt);
        F += f;
        if (f > maxf) maxf = f;
    }
    st->total_flop = F;
    int32_t* buf = (int32_t*)malloc((size_t)(maxf > 0 ? maxf : 1) * sizeof(int32_t));
    if (!buf) return ORC_ERR_MEM;
    uint64_t Z = 0;
    for (int64_t i = 0; i < M; ++i) {
        uint64_t z = orc_row_nnz_one(i, Arpt, Acol, Brpt, Bcol, buf);
        nnz_exact[i] = (int64_t)z;
        Z += z;
    }
    free(buf);
    st->out_sum = Z;
    return ORC_OK;
}

/* Exact nnz of a chosen list of rows (for spot checks of large inputs). */
int orc_rows_nnz(int64_t nrows_list, const int32_t* rows, const int32_t* Arpt, const int32_t* Acol,
                 const int32_t* Brpt, const int32_t* Bcol, int64_t* nnz, uint64_t* row_flop)
{
    uint64_t maxf = 0;
    for (int64_t s = 0; s < nrows_list; ++s) {
        uint64_t f = orc_row_flop_one(rows[s], Arpt, Acol, Brpt);
        if (row_flop) row_flop[s] = f;
        if (f > maxf) maxf = f;
    }
    int32_t* buf = (int32_t*)malloc((size_t)(maxf > 0 ? maxf : 1) * sizeof(int32_t));
    if (!buf) return ORC_ERR_MEM;
    for (int64_t s = 0; s < nrows_list; ++s)
        nnz[s] = (int64_t)orc_row_nnz_one(rows[s], Arpt, Acol, Brpt, Bcol, buf);
    free(buf);
    return ORC_OK;
}

/* ------------------------------------------ the consumer (numeric product) */

/*
 * Numeric product C = A.B by its definition, for the consumer that sizes C
 * from the predicted structure (Sec. I: the prediction exists to allocate the
 * output and balance the numeric phase).  The paper gives no numeric kernel;
 * this is the plain definition C[i][j] = sum over the stored entries (i,k,a)
 * of A and (k,j,b) of B of a*b.
 *
 * Row i is accumulated in a dense array over the N columns, the terms added
 * in storage order (A's entries in order, each named B row in order), so the
 * sum of a column is the left-to-right sum of its terms.  Beside the value
 * the oracle keeps, for each output entry, the sum of |a*b| and the number of
 * terms: the rounding error of any summation order is bounded by them.  The
 * distinct columns of the row are sorted (qsort) and written in increasing
 * order.  Duplicate entries of A or B simply contribute more terms.
 *
 * Crpt (int64[M+1]) must already hold the row offsets of C (the exact counts,
 * orc_exact, prefix-summed); Ccol/Cval/Cabs/Cterms receive rpt[M] entries.
 * Returns ORC_ERR_ARG if a row's distinct count disagrees with Crpt.
 */
int orc_spgemm(int64_t M, int64_t N, const int32_t* Arpt, const int32_t* Acol, const double* Aval,
               const int32_t* Brpt, const int32_t* Bcol, const double* Bval, const int64_t* Crpt,
               int32_t* Ccol, double* Cval, double* Cabs, int32_t* Cterms)
{
    if (M < 0 || N < 0) return ORC_ERR_ARG;
    size_t n = (size_t)(N > 0 ? N : 1);
    double* acc = (double*)calloc(n, sizeof(double));
    double* aab = (double*)calloc(n, sizeof(double));
    int32_t* terms = (int32_t*)calloc(n, sizeof(int32_t));
    int64_t* seen = (int64_t*)malloc(n * sizeof(int64_t));
    int32_t* touched = (int32_t*)malloc(n * sizeof(int32_t));
    int rc = ORC_OK;
    if (!acc || !aab || !terms || !seen || !touched) rc = ORC_ERR_MEM;
    for (size_t q = 0; rc == ORC_OK && q < n; ++q) seen[q] = -1;
    for (int64_t i = 0; rc == ORC_OK && i < M; ++i) {
        int64_t nt = 0;
        for (int64_t e = Arpt[i]; e < Arpt[i + 1]; ++e) {
            const int32_t k = Acol[e];
            const double a = Aval[e];
            for (int64_t q = Brpt[k]; q < Brpt[k + 1]; ++q) {
                const int32_t j = Bcol[q];
                const double p = a * Bval[q];
                if (seen[j] != i) {
                    seen[j] = i;
                    acc[j] = 0.0;
                    aab[j] = 0.0;
                    terms[j] = 0;
                    touched[nt++] = j;
                }
                acc[j] += p;
                aab[j] += p < 0 ? -p : p;
                terms[j] += 1;
            }
        }
        if (Crpt[i + 1] - Crpt[i] != nt) {
            rc = ORC_ERR_ARG;
            break;
        }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        for (int64_t s = 0; s < nt; ++s) {
            const int32_t j = touched[s];
            const int64_t o = Crpt[i] + s;
            Ccol[o] = j;
            Cval[o] = acc[j];
            Cabs[o] = aab[j];
            Cterms[o] = terms[j];
        }
    }
    free(acc);
    free(aab);
    free(terms);
    free(seen);
    free(touched);
    return rc;
}

/* ------------------------------- the sketch estimator of related work (KMV) */

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/*
 * The existing sampling estimator of Amossen et al. as BHash uses it (Sec. III):
 * rows of A and columns of B are each kept with probability p, every
 * intermediate product (i, j) of C' = A'B' is hashed to [0, 1), the k-th
 * smallest distinct hashed value v estimates NNZ(C') = k / v, and
 * NNZ(C) = NNZ(C') / p^2 (p taken as the realised proportions of kept rows and
 * columns).
 *
 * Definitions of this build (all from the splitmix64 stream above):
 *   row i of A kept     iff (splitmix64(seed,     i) >> 11) < T
 *   column j of B kept  iff (splitmix64(seed + 1, j) >> 11) < T
 *   hash of (i, j)      =   splitmix64(seed + 2, i * N + j) >> 11   (53 bits; value / 2^53)
 * T = floor(rate * 2^53) as for the row sampler.  Distinctness is of the
 * 53-bit hash values.  When fewer than k distinct values exist, the sample's
 * NNZ is their number (the sketch is exact).
 * Outputs: rows and columns kept, products of C', distinct hash values of C',
 * and the k-th smallest distinct value (0 when fewer than k).
 */
int orc_kmv(int64_t M, int64_t N, const int32_t* Arpt, const int32_t* Acol, const int32_t* Brpt,
            const int32_t* Bcol, uint64_t T, uint64_t seed, uint64_t k, uint64_t* rows_kept,
            uint64_t* cols_kept, uint64_t* products, uint64_t* distinct, uint64_t* kth)
{
    if (M < 0 || N < 0 || k == 0) return ORC_ERR_ARG;
    uint64_t nr = 0, nc = 0, np = 0;
    unsigned char* colk = (unsigned char*)malloc((size_t)(N > 0 ? N : 1));
    if (!colk) return ORC_ERR_MEM;
    for (int64_t j = 0; j < N; ++j) {
        colk[j] = (orc_splitmix64(seed + 1u, (uint64_t)j) >> 11) < T;
        nc += colk[j];
    }
    size_t cap = 1024, n = 0;
    uint64_t* h = (uint64_t*)malloc(cap * sizeof(uint64_t));
    if (!h) {
        free(colk);
        return ORC_ERR_MEM;
    }
    for (int64_t i = 0; i < M; ++i) {
        if (!((orc_splitmix64(seed, (uint64_t)i) >> 11) < T)) continue;
        ++nr;
        for (int64_t e = Arpt[i]; e < Arpt[i + 1]; ++e) {
            const int32_t kk = Acol[e];
            for (int64_t q = Brpt[kk]; q < Brpt[kk + 1]; ++q) {
                const int32_t j = Bcol[q];
                if (!colk[j]) continue;
                ++np;
                if (n == cap) {
                    cap *= 2;
                    uint64_t* g = (uint64_t*)realloc(h, cap * sizeof(uint64_t));
                    if (!g) {
                        free(h);
                        free(colk);
                        return ORC_ERR_MEM;
                    }
                    h = g;
                }
                h[n++] = orc_splitmix64(seed + 2u, (uint64_t)i * (uint64_t)N + (uint64_t)j) >> 11;
            }
        }
    }
    qsort(h, n, sizeof(uint64_t), cmp_u64);
    uint64_t d = 0, kv = 0;
    for (size_t s = 0; s < n; ++s) {
        if (s > 0 && h[s] == h[s - 1]) continue;
        ++d;
        if (d == k) kv = h[s];
    }
    free(h);
    free(colk);
    *rows_kept = nr;
    *cols_kept = nc;
    *products = np;
    *distinct = d;
    *kth = kv;
    return ORC_OK;
}
