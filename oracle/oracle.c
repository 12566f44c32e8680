/*
 * CPU oracle for level-synchronous breadth-first search and the local
 * sparse-matrix x sparse-vector product of the 2D algorithm.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it. It shares no code with the GPU path: it has
 * its own CSR/DCSC readers and no tables, constants or helpers in common.
 *
 * Everything here is plain, serial and written for a reader to check by
 * eye against the paper:
 *
 *   oracle_bfs      Section 2.1, Algorithm 1 (serial level-synchronous BFS)
 *                   with a FIFO queue, plus the parent rule of this build:
 *                   parent[v] = minimum id among the neighbours of v one
 *                   level closer to the root (the (select, min) semiring of
 *                   section 3.2 resolves ties to the smallest id).
 *                   level[v] = hop distance d(s, v), -1 if unreachable;
 *                   parent[s] = s; parent[v] = -1 if unreachable
 *                   (Algorithm 3's output convention).
 *
 *   oracle_spmspv   Section 4.2 ("Local Computation"): the union of the
 *                   columns A(:, k) for every k present in the frontier,
 *                   each row keeping the minimum selected value; output is
 *                   a sorted sparse vector (section 4.1). Column lookup by
 *                   binary search in the DCSC column-id array JC
 *                   (section 4.1, DCSC = IR, CP, JC).
 *
 *   oracle_check_bfs  The properties that pin a (parent, level) pair to the
 *                   definition at any size: level[s] = 0, parent[s] = s;
 *                   reached and unreached sets closed under adjacency;
 *                   |level[u] - level[v]| <= 1 on every edge; every reached
 *                   v != s has parent[v] = min{u in N(v) : level[u] =
 *                   level[v] - 1} and that set is non-empty. Together these
 *                   imply that level is the hop distance and parent follows
 *                   the minimum-id rule.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Serial FIFO BFS, Algorithm 1 order. Returns 0, or -1 on bad arguments,
 * -2 on allocation failure. parent/level are caller arrays of length n. */
int oracle_bfs(int64_t n, const int64_t *off, const int32_t *col, int32_t root,
               int32_t *parent, int32_t *level)
{
    if (n <= 0 || root < 0 || (int64_t)root >= n) return -1;
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!queue) return -2;
    for (int64_t v = 0; v < n; ++v) {
        parent[v] = -1;
        level[v] = -1;             /* the "infinity" of Algorithm 1 */
    }
    level[root] = 0;
    parent[root] = root;
    int64_t head = 0, tail = 0;
    queue[tail++] = root;
    while (head < tail) {
        const int32_t u = queue[head++];
        const int32_t next = level[u] + 1;
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            const int32_t v = col[e];
            if (level[v] == -1) {          /* first visit: distance fixed */
                level[v] = next;
                parent[v] = u;
                queue[tail++] = v;
            } else if (level[v] == next && u < parent[v]) {
                parent[v] = u;             /* smaller id one level up */
            }
        }
    }
    free(queue);
    return 0;
}

/* Sum of degrees of reached vertices (each undirected edge of the searched
 * component counted twice in a symmetric CSR). */
int64_t oracle_reached_degree_sum(int64_t n, const int64_t *off, const int32_t *level)
{
    int64_t s = 0;
    for (int64_t v = 0; v < n; ++v)
        if (level[v] >= 0) s += off[v + 1] - off[v];
    return s;
}

static int cmp_i32(const void *a, const void *b)
{
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Position of column k in JC (ascending), or -1. */
static int64_t find_column(int64_t nzc, const int32_t *jc, int32_t k)
{
    int64_t lo = 0, hi = nzc - 1;
    while (lo <= hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (jc[mid] == k) return mid;
        if (jc[mid] < k) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/*
 * out[r] = min{ val(k) : k in frontier, A(r, k) != 0 }, emitted for every r
 * with a non-empty set, ascending r. val(k) = fval[i] when fval is given,
 * else the frontier index k itself. out_idx/out_val must hold `capacity`
 * entries. Returns the output count, -1 on bad arguments, -2 on allocation
 * failure, or -(3 + needed) when capacity is too small.
 */
int64_t oracle_spmspv(int32_t nrows, int32_t ncols, int64_t nzc, const int32_t *jc,
                      const int32_t *cp, const int32_t *ir, int64_t fnnz, const int32_t *fidx,
                      const int32_t *fval, int64_t capacity, int32_t *out_idx, int32_t *out_val)
{
    if (nrows < 0 || ncols < 0 || nzc < 0 || fnnz < 0) return -1;
    int32_t *acc = (int32_t *)malloc((size_t)(nrows > 0 ? nrows : 1) * sizeof(int32_t));
    unsigned char *seen = (unsigned char *)calloc((size_t)(nrows > 0 ? nrows : 1), 1);
    int64_t touched_cap = 1024, ntouched = 0;
    int32_t *touched = (int32_t *)malloc((size_t)touched_cap * sizeof(int32_t));
    if (!acc || !seen || !touched) {
        free(acc); free(seen); free(touched);
        return -2;
    }
    for (int64_t i = 0; i < fnnz; ++i) {
        const int32_t k = fidx[i];
        const int32_t value = fval ? fval[i] : k;
        const int64_t p = find_column(nzc, jc, k);
        if (p < 0) continue;               /* empty column contributes nothing */
        for (int64_t q = cp[p]; q < cp[p + 1]; ++q) {
            const int32_t r = ir[q];
            if (!seen[r]) {
                seen[r] = 1;
                acc[r] = value;
                if (ntouched == touched_cap) {
                    touched_cap *= 2;
                    int32_t *t = (int32_t *)realloc(touched, (size_t)touched_cap * sizeof(int32_t));
                    if (!t) { free(acc); free(seen); free(touched); return -2; }
                    touched = t;
                }
                touched[ntouched++] = r;
            } else if (value < acc[r]) {
                acc[r] = value;
            }
        }
    }
    if (ntouched > capacity) {
        free(acc); free(seen); free(touched);
        return -(3 + ntouched);
    }
    qsort(touched, (size_t)ntouched, sizeof(int32_t), cmp_i32);
    for (int64_t i = 0; i < ntouched; ++i) {
        out_idx[i] = touched[i];
        out_val[i] = acc[touched[i]];
    }
    free(acc); free(seen); free(touched);
    return ntouched;
}

/*
 * Checks a (parent, level) pair against the definition. Returns 0 when all
 * properties hold, otherwise a positive code naming the first failure and
 * the offending vertex in *bad_vertex:
 *   1 root level/parent wrong, or a level-0 vertex other than the root
 *   2 level/parent reachability disagree
 *   3 edge joins reached and unreached      4 edge with |level diff| > 1
 *   5 reached vertex without a neighbour one level up
 *   6 parent is not the minimum-id neighbour one level up
 *   7 negative level other than -1 or out-of-range parent
 */
int oracle_check_bfs(int64_t n, const int64_t *off, const int32_t *col, int32_t root,
                     const int32_t *parent, const int32_t *level, int64_t *bad_vertex)
{
    *bad_vertex = -1;
    if (root < 0 || (int64_t)root >= n) return 1;
    if (level[root] != 0 || parent[root] != root) { *bad_vertex = root; return 1; }
    for (int64_t v = 0; v < n; ++v) {
        if (level[v] < -1 || parent[v] < -1 || (int64_t)parent[v] >= n) {
            *bad_vertex = v;
            return 7;
        }
        if ((level[v] == -1) != (parent[v] == -1)) { *bad_vertex = v; return 2; }
        if (level[v] == 0 && v != root) { *bad_vertex = v; return 1; }
    }
    for (int64_t v = 0; v < n; ++v) {
        int32_t best = -1;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            const int32_t u = col[e];
            if ((level[v] == -1) != (level[u] == -1)) { *bad_vertex = v; return 3; }
            if (level[v] == -1) continue;
            const int32_t d = level[v] - level[u];
            if (d > 1 || d < -1) { *bad_vertex = v; return 4; }
            if (d == 1 && (best == -1 || u < best)) best = u;
        }
        if (level[v] > 0) {
            if (best == -1) { *bad_vertex = v; return 5; }
            if (parent[v] != best) { *bad_vertex = v; return 6; }
        }
    }
    return 0;
}
