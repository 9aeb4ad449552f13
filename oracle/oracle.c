/*
 * CPU oracle for exact edit distance (Levenshtein), written from
 * "Efficient Parallel Output-Sensitive Edit Distance" (Ding, Dong, Gu, Liu,
 * Sun; ESA 2023, arXiv 2306.17461).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file.  It is used by the test suite, by the smoke check and by the
 * CPU-baseline leg of the benchmark.  It shares no code with the HIP library:
 * no headers, helpers, tables or constants.
 *
 * Conventions (one reading applied throughout):
 *   - strings are 0-based byte arrays A[0..n), B[0..m);
 *   - a grid cell (x, y) means "x chars of A and y chars of B consumed";
 *   - diagonal i = x - y;
 *   - LCP(x, y) is the length of the longest common prefix of A[x..n) and
 *     B[y..m)  (paper section 2, "Longest Common Prefix");
 *   - a frontier entry that does not exist holds ORC_NONE = -2^30, which is
 *     far enough below 0 that adding 1 never yields a valid row.
 *
 * Functions and the passage each follows:
 *   orc_dp_ed        DP recurrence of section 1 (two rows).
 *   orc_dp_matrix    the same recurrence, full (n+1)x(m+1) matrix.
 *   orc_rt_dump      R_t[i] = max{x : G[x][x-i] <= t} from the full matrix;
 *                    the BFS view of section 3.1 (cells with distance t).
 *   orc_brute_from   breadth-first search over strings, independent of the DP:
 *                    the edit-distance definition of section 2 (minimum number
 *                    of unit insertions, deletions, substitutions).
 *   orc_lcp          character loop for the LCP definition of section 2.
 *   orc_lv_naive     Algorithm 1 (section 3.1 and appendix A): rounds t, three
 *                    predecessor directions per diagonal, one LCP slide per
 *                    direction, keep the largest row.
 *   orc_hash_base    base r of the polynomial hash, from a 64-bit seed.
 *   orc_horner_table prefix table T[j] = h(A[0..jb)) of section 3.3 (the
 *                    blocked table; b = 1 gives the full table of section 3.2),
 *                    evaluated by plain Horner over every character.
 *   orc_substr_hash  h(A[l..r)) by Horner (section 2, "Hash Functions").
 *   orc_lv_omp       multicore Landau-Vishkin (Algorithm 1 with one slide per
 *                    diagonal and an 8-byte word compare); the timed CPU
 *                    baseline, checked against orc_lv_naive and orc_dp_ed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_NONE (-(1 << 30))

/* ------------------------------------------------------------------------ */
/* Section 1: the DP recurrence.                                            */
/*   G[i,0] = i, G[0,j] = j;                                                */
/*   G[i,j] = G[i-1,j-1]                 if A[i] = B[j]  (1-based)          */
/*          = 1 + min(G[i-1,j], G[i-1,j-1], G[i,j-1])  otherwise.           */
/* ------------------------------------------------------------------------ */
int64_t orc_dp_ed(const uint8_t *A, int64_t n, const uint8_t *B, int64_t m)
{
    int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return -1;
    }
    for (int64_t j = 0; j <= m; j++)
        prev[j] = j;
    for (int64_t i = 1; i <= n; i++) {
        cur[0] = i;
        for (int64_t j = 1; j <= m; j++) {
            if (A[i - 1] == B[j - 1]) {
                cur[j] = prev[j - 1];
            } else {
                int64_t best = prev[j];
                if (prev[j - 1] < best)
                    best = prev[j - 1];
                if (cur[j - 1] < best)
                    best = cur[j - 1];
                cur[j] = best + 1;
            }
        }
        int64_t *tmp = prev;
        prev = cur;
        cur = tmp;
    }
    int64_t result = prev[m];
    free(prev);
    free(cur);
    return result;
}

/* Full matrix, row-major, G[x*(m+1)+y]. */
int orc_dp_matrix(const uint8_t *A, int64_t n, const uint8_t *B, int64_t m, int32_t *G)
{
    int64_t w = m + 1;
    for (int64_t y = 0; y <= m; y++)
        G[y] = (int32_t)y;
    for (int64_t x = 1; x <= n; x++) {
        G[x * w] = (int32_t)x;
        for (int64_t y = 1; y <= m; y++) {
            if (A[x - 1] == B[y - 1]) {
                G[x * w + y] = G[(x - 1) * w + (y - 1)];
            } else {
                int32_t best = G[(x - 1) * w + y];
                if (G[(x - 1) * w + (y - 1)] < best)
                    best = G[(x - 1) * w + (y - 1)];
                if (G[x * w + (y - 1)] < best)
                    best = G[x * w + (y - 1)];
                G[x * w + y] = best + 1;
            }
        }
    }
    return 0;
}

/*
 * Frontier rows from the DP matrix.  Row t (t = 0..ED) holds 2t+1 entries for
 * diagonals i = -t..t at offset t*t; entry = max{x : 0<=x<=n, y=x-i in [0,m],
 * G[x][y] <= t}, or ORC_NONE if the diagonal has no such cell.
 * Returns ED, or -1 if the output capacity (entries) is too small.
 */
int64_t orc_rt_dump(const uint8_t *A, int64_t n, const uint8_t *B, int64_t m, int32_t *out,
                    int64_t cap)
{
    int64_t w = m + 1;
    int32_t *G = (int32_t *)malloc(sizeof(int32_t) * (size_t)((n + 1) * w));
    if (!G)
        return -1;
    orc_dp_matrix(A, n, B, m, G);
    int64_t ed = G[n * w + m];
    if ((ed + 1) * (ed + 1) > cap) {
        free(G);
        return -1;
    }
    for (int64_t t = 0; t <= ed; t++) {
        for (int64_t i = -t; i <= t; i++) {
            int32_t best = ORC_NONE;
            for (int64_t x = 0; x <= n; x++) {
                int64_t y = x - i;
                if (y < 0 || y > m)
                    continue;
                if (G[x * w + y] <= t)
                    best = (int32_t)x;
            }
            out[t * t + (i + t)] = best;
        }
    }
    free(G);
    return ed;
}

/* ------------------------------------------------------------------------ */
/* Brute force: BFS in string space from A.  Every string over {0..sigma-1} */
/* of length <= maxlen is a vertex; its neighbours are the strings one      */
/* insertion, deletion or substitution away (section 2 definition).         */
/* Vertex index of a string s of length l: off[l] + value of s in base      */
/* sigma (most significant digit first).                                    */
/* dist[] receives the distance from A to every vertex (-1 = unreached).    */
/* Returns the number of vertices, or -1 on bad arguments.                  */
/* ------------------------------------------------------------------------ */
static int64_t brute_index(const uint8_t *s, int l, int sigma, const int64_t *off)
{
    int64_t v = 0;
    for (int i = 0; i < l; i++)
        v = v * sigma + s[i];
    return off[l] + v;
}

int64_t orc_brute_count(int sigma, int maxlen)
{
    int64_t total = 0, p = 1;
    for (int l = 0; l <= maxlen; l++) {
        total += p;
        p *= sigma;
    }
    return total;
}

int64_t orc_brute_from(const uint8_t *A, int n, int sigma, int maxlen, int32_t *dist)
{
    if (sigma < 1 || sigma > 8 || maxlen < 0 || maxlen > 12 || n > maxlen)
        return -1;
    int64_t off[16];
    int64_t p = 1;
    off[0] = 0;
    for (int l = 0; l <= maxlen; l++) {
        off[l + 1] = off[l] + p;
        p *= sigma;
    }
    int64_t total = off[maxlen + 1];
    for (int64_t v = 0; v < total; v++)
        dist[v] = -1;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)total);
    if (!queue)
        return -1;
    int64_t head = 0, tail = 0;
    int64_t src = brute_index(A, n, sigma, off);
    dist[src] = 0;
    queue[tail++] = src;
    uint8_t s[16], u[16];
    while (head < tail) {
        int64_t v = queue[head++];
        /* decode v -> (l, s) */
        int l = 0;
        while (off[l + 1] <= v)
            l++;
        int64_t val = v - off[l];
        for (int i = l - 1; i >= 0; i--) {
            s[i] = (uint8_t)(val % sigma);
            val /= sigma;
        }
        int32_t d = dist[v] + 1;
        /* deletions */
        for (int pos = 0; pos < l; pos++) {
            int k = 0;
            for (int i = 0; i < l; i++)
                if (i != pos)
                    u[k++] = s[i];
            int64_t nv = brute_index(u, l - 1, sigma, off);
            if (dist[nv] < 0) {
                dist[nv] = d;
                queue[tail++] = nv;
            }
        }
        /* insertions */
        if (l < maxlen) {
            for (int pos = 0; pos <= l; pos++) {
                for (int c = 0; c < sigma; c++) {
                    int k = 0;
                    for (int i = 0; i < pos; i++)
                        u[k++] = s[i];
                    u[k++] = (uint8_t)c;
                    for (int i = pos; i < l; i++)
                        u[k++] = s[i];
                    int64_t nv = brute_index(u, l + 1, sigma, off);
                    if (dist[nv] < 0) {
                        dist[nv] = d;
                        queue[tail++] = nv;
                    }
                }
            }
        }
        /* substitutions */
        for (int pos = 0; pos < l; pos++) {
            for (int c = 0; c < sigma; c++) {
                if (c == s[pos])
                    continue;
                memcpy(u, s, (size_t)l);
                u[pos] = (uint8_t)c;
                int64_t nv = brute_index(u, l, sigma, off);
                if (dist[nv] < 0) {
                    dist[nv] = d;
                    queue[tail++] = nv;
                }
            }
        }
    }
    free(queue);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Section 2: LCP(A, B, x, y) by a character loop.                          */
/* ------------------------------------------------------------------------ */
int64_t orc_lcp(const uint8_t *A, int64_t n, const uint8_t *B, int64_t m, int64_t x, int64_t y)
{
    int64_t l = 0;
    while (x + l < n && y + l < m && A[x + l] == B[y + l])
        l++;
    return l;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (section 3.1, appendix A), sequential and literal:           */
/*   f_0[0] = LCP(0, 0);                                                    */
/*   while the target cell (n, m) is not on the frontier:                   */
/*     t = t + 1;                                                           */
/*     for every diagonal i in [-t, t]:                                     */
/*       f_t[i] = f_{t-1}[i];                                               */
/*       for each predecessor direction (dx, dy) in {(0,1), (1,0), (1,1)}:  */
/*         j = i - dx + dy;  if |j| <= t-1 and f_{t-1}[j] exists:           */
/*           x = f_{t-1}[j] + dx;  y = x - i;                               */
/*           x = x + LCP(x, y);                                             */
/*           f_t[i] = max(f_t[i], x).                                       */
/* Readings where the listing is silent:                                    */
/*   - a diagonal that did not exist in round t-1 starts at ORC_NONE;       */
/*   - only diagonals with a grid cell, i in [max(-t,-m), min(t,n)], are    */
/*     processed; the rest stay ORC_NONE;                                   */
/*   - a candidate beyond the grid is clamped to the last cell of its       */
/*     diagonal: x = min(x, n, m + i)  (adjacent DP cells differ by <= 1,   */
/*     so the clamped cell is still within t edits);                        */
/*   - the target test f_t[n-m] = n applies once diagonal n-m exists;       */
/*   - with k_max >= 0 the search stops after round k_max and returns       */
/*     k_max + 1 when the target was not reached.                           */
/* dump (optional): row t at offset t*t, 2t+1 entries for i = -t..t.        */
/* Returns ED, k_max + 1, or -1 (allocation or dump capacity failure, or a  */
/* search longer than max(n, m) rounds, which cannot happen).               */
/* ------------------------------------------------------------------------ */
int64_t orc_lv_naive(const uint8_t *A, int64_t n, const uint8_t *B, int64_t m, int64_t k_max,
                     int32_t *dump, int64_t dump_cap)
{
    int64_t K = (n > m ? n : m) + 1; /* diagonals -K..K are enough: ED <= max(n,m) */
    int32_t *fp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * K + 1));
    int32_t *fc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * K + 1));
    if (!fp || !fc) {
        free(fp);
        free(fc);
        return -1;
    }
    for (int64_t i = 0; i < 2 * K + 1; i++) {
        fp[i] = ORC_NONE;
        fc[i] = ORC_NONE;
    }
    int64_t t = 0;
    fp[K + 0] = (int32_t)orc_lcp(A, n, B, m, 0, 0);
    if (dump) {
        if (dump_cap < 1)
            goto fail;
        dump[0] = fp[K];
    }
    const int64_t target = n - m;
    for (;;) {
        int64_t at = target < 0 ? -target : target;
        if (t >= at && fp[K + target] == n)
            break;
        if (k_max >= 0 && t >= k_max) {
            t = k_max + 1;
            break;
        }
        if (t >= K - 1) /* ED <= max(n, m): a longer search is a bug */
            goto fail;
        t++;
        int64_t lo = -t > -m ? -t : -m;
        int64_t hi = t < n ? t : n;
        for (int64_t i = -t; i <= t; i++)
            fc[K + i] = ORC_NONE;
        for (int64_t i = lo; i <= hi; i++) {
            int64_t best = (i >= -(t - 1) && i <= t - 1) ? fp[K + i] : ORC_NONE;
            static const int dirs[3][2] = {{0, 1}, {1, 0}, {1, 1}};
            for (int d = 0; d < 3; d++) {
                int64_t dx = dirs[d][0], dy = dirs[d][1];
                int64_t j = i - dx + dy;
                if (j < -(t - 1) || j > t - 1)
                    continue;
                if (fp[K + j] == ORC_NONE)
                    continue;
                int64_t x = fp[K + j] + dx;
                if (x > n)
                    x = n;
                if (x > m + i)
                    x = m + i;
                int64_t y = x - i;
                x = x + orc_lcp(A, n, B, m, x, y);
                if (x > best)
                    best = x;
            }
            fc[K + i] = (int32_t)best;
        }
        int32_t *tmp = fp;
        fp = fc;
        fc = tmp;
        if (dump) {
            if ((t + 1) * (t + 1) > dump_cap)
                goto fail;
            for (int64_t i = -t; i <= t; i++)
                dump[t * t + (i + t)] = fp[K + i];
        }
    }
    free(fp);
    free(fc);
    return t;
fail:
    free(fp);
    free(fc);
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Section 2 "Hash Functions": h(S) = sum_i S[i] * r^(|S|-1-i) mod P with   */
/* P = 2^61 - 1; characters enter with their byte values 0..255.            */
/* The base r comes from a 64-bit seed through one splitmix64 output        */
/* (Steele, Lea, Flood 2014; constants as published by Vigna):              */
/*   z = seed + 0x9E3779B97F4A7C15;                                         */
/*   z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9;                              */
/*   z = (z ^ (z >> 27)) * 0x94D049BB133111EB;                              */
/*   z = z ^ (z >> 31);                                                     */
/* then r = 2^20 + (z mod (P - 2^21)), i.e. r in [2^20, P - 2^20).          */
/* ------------------------------------------------------------------------ */
#define ORC_P ((((uint64_t)1) << 61) - 1)

uint64_t orc_hash_base(uint64_t seed)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    uint64_t span = ORC_P - (((uint64_t)1) << 21);
    return (((uint64_t)1) << 20) + (z % span);
}

static uint64_t orc_mulmod(uint64_t a, uint64_t b)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    return (uint64_t)(p % ORC_P);
}

/* h(A[l..r)) by Horner: h = h * r + A[i]. */
uint64_t orc_substr_hash(const uint8_t *A, int64_t l, int64_t r, uint64_t base)
{
    uint64_t h = 0;
    for (int64_t i = l; i < r; i++)
        h = (orc_mulmod(h, base) + A[i]) % ORC_P;
    return h;
}

/* Section 3.3 table: T[0] = 0 and T[j] = h(A[0..jb)) for j = 1..floor(n/b). */
int orc_horner_table(const uint8_t *A, int64_t n, int64_t b, uint64_t base, uint64_t *T)
{
    if (b < 1)
        return -1;
    uint64_t h = 0;
    T[0] = 0;
    int64_t nb = n / b;
    for (int64_t j = 1; j <= nb; j++) {
        for (int64_t i = (j - 1) * b; i < j * b; i++)
            h = (orc_mulmod(h, base) + A[i]) % ORC_P;
        T[j] = h;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Multicore Landau-Vishkin: the timed CPU baseline.                        */
/* Each round is an OpenMP parallel loop over the diagonals.  The three     */
/* slides of Algorithm 1 are replaced by one slide from the largest clamped */
/* candidate: sliding along a diagonal is monotone and a slide from a lower */
/* start that passes a higher start ends where that one ends, so the max of */
/* three slides equals one slide of the max (checked against orc_lv_naive). */
/* The LCP compares 8-byte words (memcpy loads, XOR, count trailing zero    */
/* bits) after the leading 8 characters, the shortcut of section 5.1.       */
/* Returns ED (or k_max + 1), -1 on allocation failure or a search longer   */
/* than max(n, m) rounds.                                                   */
/* ------------------------------------------------------------------------ */
static int64_t omp_lcp(const uint8_t *A, int64_t n, const uint8_t *B, int64_t m, int64_t x,
                       int64_t y)
{
    int64_t lim = (n - x) < (m - y) ? (n - x) : (m - y);
    int64_t l = 0;
    while (l + 8 <= lim) {
        uint64_t a, b;
        memcpy(&a, A + x + l, 8);
        memcpy(&b, B + y + l, 8);
        uint64_t d = a ^ b;
        if (d)
            return l + (__builtin_ctzll(d) >> 3);
        l += 8;
    }
    while (l < lim && A[x + l] == B[y + l])
        l++;
    return l;
}

int64_t orc_lv_omp(const uint8_t *A, int64_t n, const uint8_t *B, int64_t m, int64_t k_max,
                   int threads)
{
    int64_t K = (n > m ? n : m) + 1;
    int32_t *fp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * K + 3));
    int32_t *fc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * K + 3));
    if (!fp || !fc) {
        free(fp);
        free(fc);
        return -1;
    }
    /* index i maps to i + K + 1 so that i-1 and i+1 stay in range */
    int64_t off = K + 1;
    fp[off - 1] = ORC_NONE;
    fp[off + 1] = ORC_NONE;
    fc[off - 1] = ORC_NONE;
    fc[off + 1] = ORC_NONE;
    fp[off] = (int32_t)omp_lcp(A, n, B, m, 0, 0);
#ifdef _OPENMP
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    int64_t t = 0;
    const int64_t target = n - m;
    for (;;) {
        int64_t at = target < 0 ? -target : target;
        if (t >= at && fp[off + target] == n)
            break;
        if (k_max >= 0 && t >= k_max) {
            t = k_max + 1;
            break;
        }
        if (t >= K - 1) { /* ED <= max(n, m): a longer search is a bug */
            t = -1;
            break;
        }
        t++;
        int64_t lo = -t > -m ? -t : -m;
        int64_t hi = t < n ? t : n;
        /* Entries never written must read as ORC_NONE.  Round t reads fp at
         * -t-1..t+1 and writes fc inside [-t, t]; marking +-t and +-(t+1)
         * in both buffers each round initialises every index before its
         * first read. */
        fc[off - t - 1] = ORC_NONE;
        fc[off + t + 1] = ORC_NONE;
        fc[off - t] = ORC_NONE;
        fc[off + t] = ORC_NONE;
        fp[off - t - 1] = ORC_NONE;
        fp[off + t + 1] = ORC_NONE;
        fp[off - t] = ORC_NONE;
        fp[off + t] = ORC_NONE;
#pragma omp parallel for schedule(static)
        for (int64_t i = lo; i <= hi; i++) {
            int64_t c = ORC_NONE;
            int64_t v;
            v = fp[off + i];
            if (v != ORC_NONE && v + 1 > c)
                c = v + 1;
            v = fp[off + i - 1];
            if (v != ORC_NONE && v + 1 > c)
                c = v + 1;
            v = fp[off + i + 1];
            if (v != ORC_NONE && v > c)
                c = v;
            if (c == ORC_NONE) {
                fc[off + i] = ORC_NONE;
                continue;
            }
            if (c > n)
                c = n;
            if (c > m + i)
                c = m + i;
            fc[off + i] = (int32_t)(c + omp_lcp(A, n, B, m, c, c - i));
        }
        int32_t *tmp = fp;
        fp = fc;
        fc = tmp;
    }
    free(fp);
    free(fc);
    return t;
}

int orc_omp_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
