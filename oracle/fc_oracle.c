/*
 * fc_oracle.c -- plain, slow, obviously correct CPU reference for exact
 * counting queries over a complete categorical database.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may
 * include, link, load or call this file.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark use it.  It shares no
 * code, header, table or constant with the GPU path.
 *
 * Paper: Karan, Eichhorn, Hurlburt, Iraci, Zola, "Fast Counting in Machine
 * Learning Applications" (UAI 2018, arXiv 1804.04640).
 *
 * Conventions (readings of the paper, listed in the design notes):
 *   - D is stored column-major: column v is m bytes, D[v*m + p] is the
 *     0-based state of variable v in instance p.  The paper numbers states
 *     1..r_i (Section 2); state s here is the paper's state s+1.
 *   - A query is an ordered list of distinct variables vars[0..k-1].  For
 *     Query(X_i, Pa) the child X_i is last.  The dense table index is the
 *     mixed-radix number with vars[0] most significant and the child least
 *     significant, so row j (a parent configuration) is the contiguous
 *     slice [j*r_i, (j+1)*r_i) -- the MSD radix digit order of Section 3.3.
 *   - Floating point is IEEE binary64 throughout; every sum uses Neumaier
 *     compensated summation in the order the terms are enumerated.
 *
 * Every function is "parity pinned" by the CPU test-suite (worked example,
 * brute force, entropy and Polya-urn identities, library routines); see the
 * header comment of each function for the passage it follows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)

/* ------------------------------------------------------------------ */
/* Compensated (Neumaier) summation in binary64.                       */
/* ------------------------------------------------------------------ */
typedef struct {
    double s, c;
} orc_acc;

static void acc_add(orc_acc *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double acc_get(const orc_acc *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Query validation shared by the counting functions of this file.     */
/* ------------------------------------------------------------------ */
static int check_query(int32_t n, const uint8_t *arity, const int32_t *vars,
                       int32_t k)
{
    if (k < 1)
        return ORC_EINVAL;
    for (int32_t t = 0; t < k; ++t) {
        if (vars[t] < 0 || vars[t] >= n)
            return ORC_EINVAL;
        if (arity[vars[t]] == 0)
            return ORC_EINVAL;
        for (int32_t u = 0; u < t; ++u)
            if (vars[u] == vars[t])
                return ORC_EINVAL; /* a query is a *set* of variables */
    }
    return ORC_OK;
}

/*
 * Number of cells of the contingency table of a query: r_i * q_i with
 * q_i the product of the parents' arities (Section 2, after Eq. (1)).
 * Returns -1 on an invalid query.
 */
int64_t orc_table_cells(const uint8_t *arity, int32_t n, const int32_t *vars,
                        int32_t k)
{
    if (check_query(n, arity, vars, k) != ORC_OK)
        return -1;
    int64_t c = 1;
    for (int32_t t = 0; t < k; ++t)
        c *= (int64_t)arity[vars[t]];
    return c;
}

/*
 * Full contingency table of a query (Section 2): cell
 * (s_0, ..., s_{k-1}) holds the number of instances p with
 * D[vars[t]][p] == s_t for every t.  One pass over the instances; each
 * instance adds one to the cell its states name.  Both the Bitmap
 * strategy (Section 3.2) and the Radix strategy (Section 3.3) reach exactly
 * these numbers; this is the definition, not either algorithm.
 *
 * table must hold `cells` int64 entries; it is overwritten.
 * Returns 0, or -1 for an invalid query, a cells mismatch or a state that is
 * not below its variable's arity (the database must be complete).
 */
int orc_count(const uint8_t *cols, int64_t m, int32_t n, const uint8_t *arity,
              const int32_t *vars, int32_t k, int64_t *table, int64_t cells)
{
    int64_t want = orc_table_cells(arity, n, vars, k);
    if (want < 0 || want != cells || m < 0)
        return ORC_EINVAL;
    memset(table, 0, (size_t)cells * sizeof(int64_t));
    for (int64_t p = 0; p < m; ++p) {
        int64_t idx = 0;
        for (int32_t t = 0; t < k; ++t) {
            int32_t v = vars[t];
            uint8_t s = cols[(int64_t)v * m + p];
            if (s >= arity[v])
                return ORC_EINVAL;
            idx = idx * arity[v] + s;
        }
        table[idx] += 1;
    }
    return ORC_OK;
}

/*
 * Single-assignment count Count((X_a = x_a) AND (X_b = x_b) AND ...)
 * (Section 2; the single-path specialisation closing Section 3.3).
 * Returns the count, or -1 for an invalid query or a state out of range.
 */
int64_t orc_count_assignment(const uint8_t *cols, int64_t m, int32_t n,
                             const uint8_t *arity, const int32_t *vars,
                             const uint8_t *states, int32_t k)
{
    if (check_query(n, arity, vars, k) != ORC_OK || m < 0)
        return -1;
    for (int32_t t = 0; t < k; ++t)
        if (states[t] >= arity[vars[t]])
            return -1;
    int64_t cnt = 0;
    for (int64_t p = 0; p < m; ++p) {
        int match = 1;
        for (int32_t t = 0; t < k && match; ++t)
            match = cols[(int64_t)vars[t] * m + p] == states[t];
        cnt += match;
    }
    return cnt;
}

/* N_ij: the sum of row j of a q x r table. */
static int64_t row_sum(const int64_t *T, int64_t j, int32_t r)
{
    int64_t s = 0;
    for (int32_t k = 0; k < r; ++k)
        s += T[j * r + k];
    return s;
}

/*
 * Log-likelihood of Eq. (1), in bits as in the function object of Fig. 2:
 *   LL = sum_j sum_k N_ijk * log2(N_ijk / N_ij),
 * summed over the cells with N_ijk > 0 only (zero counts are never emitted,
 * Section 2).  T is the q x r table of Query(X_i, Pa), child fastest.
 */
double orc_ll(const int64_t *T, int64_t q, int32_t r)
{
    orc_acc a = {0.0, 0.0};
    for (int64_t j = 0; j < q; ++j) {
        int64_t nij = row_sum(T, j, r);
        for (int32_t k = 0; k < r; ++k) {
            int64_t nijk = T[j * r + k];
            if (nijk > 0)
                acc_add(&a, (double)nijk * log2((double)nijk / (double)nij));
        }
    }
    return acc_get(&a);
}

/*
 * MDL family score (the paper's solver uses MDL, Section 4.2, citing
 * Schwarz 1978; the formula itself is not printed).  Reading used here, to
 * be minimised:
 *   MDL = -LL + (1/2) * log2(m) * q_i * (r_i - 1),
 * with LL in bits, m the number of instances and q_i the full product of
 * the parents' arities (Section 2).
 */
double orc_mdl(const int64_t *T, int64_t q, int32_t r)
{
    int64_t m = 0;
    for (int64_t j = 0; j < q; ++j)
        m += row_sum(T, j, r);
    double penalty = 0.5 * log2((double)m) * (double)q * (double)(r - 1);
    orc_acc a = {0.0, 0.0};
    acc_add(&a, -orc_ll(T, q, r));
    acc_add(&a, penalty);
    return acc_get(&a);
}

/*
 * BDeu family score (Dirichlet priors with the product of gamma functions,
 * Section 3.1, citing Cooper 1992; Section 4.2).  Reading used here, in
 * nats, to be maximised, with equivalent sample size ess,
 * a_j = ess / q and a_jk = ess / (r q):
 *   sum_{j: N_ij > 0}  [lnG(a_j)  - lnG(a_j  + N_ij)]
 * + sum_{jk: N_ijk > 0}[lnG(a_jk + N_ijk) - lnG(a_jk)].
 * Configurations that never occur contribute exactly zero, which is why only
 * the non-zero part of the table has to be streamed (Section 2).
 */
double orc_bdeu(const int64_t *T, int64_t q, int32_t r, double ess)
{
    double aj = ess / (double)q;
    double ajk = ess / ((double)r * (double)q);
    double lg_aj = lgamma(aj), lg_ajk = lgamma(ajk);
    orc_acc a = {0.0, 0.0};
    for (int64_t j = 0; j < q; ++j) {
        int64_t nij = row_sum(T, j, r);
        if (nij == 0)
            continue;
        acc_add(&a, lg_aj);
        acc_add(&a, -lgamma(aj + (double)nij));
        for (int32_t k = 0; k < r; ++k) {
            int64_t nijk = T[j * r + k];
            if (nijk > 0) {
                acc_add(&a, lgamma(ajk + (double)nijk));
                acc_add(&a, -lg_ajk);
            }
        }
    }
    return acc_get(&a);
}

/*
 * Mutual information between the child and the joint state of the other
 * query variables (a constraint test in BN learning, Section 1), in nats:
 *   MI = sum_{jk: N_ijk > 0} (N_ijk / m) * ln(m * N_ijk / (N_ij * N_.k)),
 * with N_.k the count of child state k over all rows of the table.
 */
double orc_mi(const int64_t *T, int64_t q, int32_t r)
{
    int64_t *nk = (int64_t *)calloc((size_t)r, sizeof(int64_t));
    if (!nk)
        return NAN;
    int64_t m = 0;
    for (int64_t j = 0; j < q; ++j)
        for (int32_t k = 0; k < r; ++k) {
            nk[k] += T[j * r + k];
            m += T[j * r + k];
        }
    orc_acc a = {0.0, 0.0};
    for (int64_t j = 0; j < q; ++j) {
        int64_t nij = row_sum(T, j, r);
        for (int32_t k = 0; k < r; ++k) {
            int64_t nijk = T[j * r + k];
            if (nijk > 0) {
                /* ln(m N_ijk / (N_ij N_k)) as ln(1 + x), x formed from the
                 * exact integer difference m N_ijk - N_ij N_k (both below
                 * 2^62): a ratio rounded first would carry an absolute
                 * error near 1e-16 into every term, which is not small
                 * against a mutual information close to 0 */
                int64_t den = nij * nk[k];
                int64_t num = m * nijk - den;
                double x = (double)num / (double)den;
                acc_add(&a, ((double)nijk / (double)m) * log1p(x));
            }
        }
    }
    free(nk);
    return acc_get(&a);
}

/*
 * All-pairs co-occurrence counts of binary items (association rule mining,
 * Section 4.3): gram[a*n + b] = Count((X_a = 1) AND (X_b = 1)), the diagonal
 * being the support count of each single item.  cols holds n binary columns
 * of m bytes (states 0/1).  Rows are visited in blocks; for each instance the
 * items present are listed and every pair of them is counted once.
 * gram must hold n*n int64 entries; it is overwritten.  Returns 0 or -1.
 */
int orc_gram(const uint8_t *cols, int64_t m, int32_t n, int64_t *gram)
{
    if (n < 1 || m < 0)
        return ORC_EINVAL;
    memset(gram, 0, (size_t)n * (size_t)n * sizeof(int64_t));
    const int64_t B = 4096;
    int32_t *lst = (int32_t *)malloc((size_t)B * (size_t)n * sizeof(int32_t));
    int32_t *len = (int32_t *)malloc((size_t)B * sizeof(int32_t));
    if (!lst || !len) {
        free(lst);
        free(len);
        return ORC_EINVAL;
    }
    for (int64_t p0 = 0; p0 < m; p0 += B) {
        int64_t nb = (m - p0 < B) ? (m - p0) : B;
        memset(len, 0, (size_t)nb * sizeof(int32_t));
        for (int32_t a = 0; a < n; ++a) {
            const uint8_t *col = cols + (int64_t)a * m + p0;
            for (int64_t i = 0; i < nb; ++i) {
                if (col[i] > 1) {
                    free(lst);
                    free(len);
                    return ORC_EINVAL;
                }
                if (col[i])
                    lst[i * n + len[i]++] = a;
            }
        }
        for (int64_t i = 0; i < nb; ++i) {
            const int32_t *l = lst + i * n;
            for (int32_t x = 0; x < len[i]; ++x)
                for (int32_t y = x; y < len[i]; ++y)
                    gram[(int64_t)l[x] * n + l[y]] += 1;
        }
    }
    for (int32_t a = 0; a < n; ++a)
        for (int32_t b = a + 1; b < n; ++b)
            gram[(int64_t)b * n + a] = gram[(int64_t)a * n + b];
    free(lst);
    free(len);
    return ORC_OK;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/*
 * Sparse table of a query (Section 2; only configurations that occur, at
 * most min(q_i r_i, m) of them, Section 3.2): the mixed-radix key of every
 * instance (first variable most significant), sorted, and each run of equal
 * keys counted.  keys_out and counts_out must hold m entries.  Returns the
 * number of distinct keys, or -1 (invalid query, state out of range, or a
 * key space of 2^63 or more).
 */
int64_t orc_count_sparse(const uint8_t *cols, int64_t m, int32_t n,
                         const uint8_t *arity, const int32_t *vars, int32_t k,
                         int64_t *keys_out, int64_t *counts_out)
{
    if (check_query(n, arity, vars, k) != ORC_OK || m < 0)
        return -1;
    double space = 1.0;
    for (int32_t t = 0; t < k; ++t)
        space *= (double)arity[vars[t]];
    if (space >= 9.2e18)
        return -1;
    int64_t *key = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!key)
        return -1;
    for (int64_t p = 0; p < m; ++p) {
        int64_t idx = 0;
        for (int32_t t = 0; t < k; ++t) {
            int32_t v = vars[t];
            uint8_t s = cols[(int64_t)v * m + p];
            if (s >= arity[v]) {
                free(key);
                return -1;
            }
            idx = idx * arity[v] + s;
        }
        key[p] = idx;
    }
    qsort(key, (size_t)m, sizeof(int64_t), cmp_i64);
    int64_t nd = 0;
    for (int64_t p = 0; p < m; ++p) {
        if (nd > 0 && keys_out[nd - 1] == key[p]) {
            counts_out[nd - 1] += 1;
        } else {
            keys_out[nd] = key[p];
            counts_out[nd] = 1;
            ++nd;
        }
    }
    free(key);
    return nd;
}
