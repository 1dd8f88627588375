/*
 * simplex_oracle.c -- plain, slow, single-threaded CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it is used by tests/, by __graft_entry__.smoke() and by the
 * cpu_baseline leg of bench.py, and by nothing else.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * What it computes (the per-element operations that the block-space map H
 * and the bounding-box map drive), written as their plain definitions:
 *
 *   Domain (Section 1, Eq. 1): the discrete orthogonal m-simplex
 *       Delta_n^m = { x in Z_+^m : 0 <= x_i <= n, x_1 + ... + x_m <= n },
 *   which has C(n+m, m) elements.  (The volume formula of Section 2,
 *   eq_volume, gives C(n+m-1, m) because there n counts cells along an
 *   edge; an edge of Delta_n^m holds n+1 cells, hence the index shift.)
 *
 *   Storage: the (n+1)^m bounding box, row-major with x_1 fastest, so the
 *   element x lives at linear index  i(x) = sum_k x_k (n+1)^(k-1).
 *   Cells outside Delta_n^m are never read as data and never written.
 *
 *   Operations (the test kernels of Section 5.1, Table tab:tests, plus a
 *   hit counter and a coordinate hash; the EDM test is oracle_edm below):
 *     MAP    -- visit every element, write nothing.
 *     ACCUM  -- out[i] = in[i] + 1  (uint32, wrapping mod 2^32).
 *     HITS   -- out[i] = out[i] + 1 (uint32): counts how often each element
 *               is visited; an exactly-once walk leaves +1 on Delta only.
 *     HASH   -- out[i] = hash32(x_1..x_m) (uint32), defined below.
 *     CA2    -- one step of Conway's Life (birth on 3, survival on 2 or 3
 *               live neighbours) over the Moore 8-neighbourhood, on uint8
 *               cells; neighbours outside Delta_n^2 count as dead.
 *     CA3    -- one step of the 3-D rule B6/S567 over the 26-neighbourhood,
 *               uint8 cells, neighbours outside Delta_n^3 count as dead.
 *   A cell is alive iff its byte equals 1; CA inputs on Delta are 0 or 1.
 *   The paper's 2-D automaton uses a periodic boundary and its 3-D one
 *   "fixed dead cells" without naming a rule (Section 5.1); here both are
 *   read as: every cell of the simplex is updated and cells outside it are
 *   dead.
 *
 *   hash32 (not in the paper; project-defined): FNV-1a over the 32-bit
 *   words x_1, ..., x_m (offset basis 0x811C9DC5, prime 0x01000193),
 *   followed by the MurmurHash3 32-bit finaliser fmix32.
 *
 * Enumeration follows Eq. 1 directly: nested loops, x_m outermost and x_1
 * innermost, each upper bound being n minus the coordinates already fixed.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

enum { OR_MAP = 0, OR_ACCUM = 1, OR_HITS = 2, OR_HASH = 3, OR_CA2 = 4, OR_CA3 = 5 };
enum { OR_OK = 0, OR_EINVAL = -1 };

/* ---- EDM (Section 5.1, Table tab:tests, test 3) ------------------------------
 *
 * The Euclidean distance matrix on the 2-simplex: the element at location
 * (i, j) holds the distance d(p_i, p_j) between two points of a set
 * p_0 .. p_n.  The paper does not fix the point dimension or the
 * placement of (i, j) in Delta_n^2; read here as: points in R^3, and the
 * element x = (x_1, x_2) holds the pair (i, j) = (x_1, n - x_2), so that
 * x_1 + x_2 <= n is exactly i <= j (the upper triangle with its diagonal,
 * the diagonal being x_1 + x_2 = n).  The oracle evaluates the definition
 * sqrt(sum_k (p_i[k] - p_j[k])^2) in double precision from the float
 * coordinates; out is a double (n+1)^2 box, written on Delta_n^2 only.
 */
int oracle_edm(int64_t n, const float *pts, double *out, int64_t *visited);

/* ---- hash32 ------------------------------------------------------------ */

uint32_t oracle_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

uint32_t oracle_fnv1a_words(int m, const uint32_t *x)
{
    uint32_t h = 0x811C9DC5u;
    for (int k = 0; k < m; ++k) {
        h ^= x[k];
        h *= 0x01000193u;
    }
    return h;
}

uint32_t oracle_hash32(int m, const uint32_t *x)
{
    return oracle_fmix32(oracle_fnv1a_words(m, x));
}

/* ---- domain helpers ------------------------------------------------------ */

/* i(x) = sum_k x_k (n+1)^(k-1), x_1 fastest. */
static int64_t lin_index(int m, int64_t n, const int64_t *x)
{
    int64_t i = 0, stride = 1;
    for (int k = 0; k < m; ++k) {
        i += x[k] * stride;
        stride *= (n + 1);
    }
    return i;
}

/* Eq. 1 membership test. */
static int in_simplex(int m, int64_t n, const int64_t *x)
{
    int64_t s = 0;
    for (int k = 0; k < m; ++k) {
        if (x[k] < 0 || x[k] > n) return 0;
        s += x[k];
    }
    return s <= n;
}

/* Number of live cells among the 3^m - 1 neighbours of x that lie in the
 * simplex (neighbours outside it are dead). */
static int live_neighbours(int m, int64_t n, const uint8_t *in, const int64_t *x)
{
    int count = 0;
    int ncomb = 1;
    for (int k = 0; k < m; ++k) ncomb *= 3;
    for (int c = 0; c < ncomb; ++c) {
        int64_t y[4];
        int t = c, zero = 1;
        for (int k = 0; k < m; ++k) {
            int d = t % 3 - 1;
            t /= 3;
            if (d != 0) zero = 0;
            y[k] = x[k] + d;
        }
        if (zero) continue;
        if (!in_simplex(m, n, y)) continue;
        if (in[lin_index(m, n, y)] == 1) ++count;
    }
    return count;
}

/* Next state of cell x under the rule of the given automaton op. */
static uint8_t ca_next(int op, int m, int64_t n, const uint8_t *in, const int64_t *x)
{
    int alive = in[lin_index(m, n, x)] == 1;
    int c = live_neighbours(m, n, in, x);
    if (op == OR_CA2) /* B3/S23 */
        return (uint8_t)(alive ? (c == 2 || c == 3) : (c == 3));
    /* OR_CA3: B6/S567 */
    return (uint8_t)(alive ? (c >= 5 && c <= 7) : (c == 6));
}

/* ---- per-element operation ---------------------------------------------- */

static void apply_one(int op, int m, int64_t n, const void *in, void *out,
                      const int64_t *x)
{
    int64_t i = lin_index(m, n, x);
    switch (op) {
    case OR_MAP:
        break;
    case OR_ACCUM:
        ((uint32_t *)out)[i] = ((const uint32_t *)in)[i] + 1u;
        break;
    case OR_HITS:
        ((uint32_t *)out)[i] += 1u;
        break;
    case OR_HASH: {
        uint32_t w[4];
        for (int k = 0; k < m; ++k) w[k] = (uint32_t)x[k];
        ((uint32_t *)out)[i] = oracle_hash32(m, w);
        break;
    }
    case OR_CA2:
    case OR_CA3:
        ((uint8_t *)out)[i] = ca_next(op, m, n, (const uint8_t *)in, x);
        break;
    }
}

static int check_args(int m, int64_t n, int op, const void *in, void *out)
{
    if (m < 2 || m > 4 || n < 0) return OR_EINVAL;
    if (op < OR_MAP || op > OR_CA3) return OR_EINVAL;
    if (op == OR_CA2 && m != 2) return OR_EINVAL;
    if (op == OR_CA3 && m != 3) return OR_EINVAL;
    if ((op == OR_ACCUM || op == OR_CA2 || op == OR_CA3) && in == NULL) return OR_EINVAL;
    if (op != OR_MAP && out == NULL) return OR_EINVAL;
    if ((op == OR_CA2 || op == OR_CA3) && in == out) return OR_EINVAL;
    return OR_OK;
}

/* Walk Delta_n^m with nested loops (x_m outermost, x_1 innermost) and apply
 * op to every element.  *visited receives the number of elements visited,
 * which must equal C(n+m, m).  Returns 0, or OR_EINVAL on bad arguments. */
int oracle_apply(int m, int64_t n, int op, const void *in, void *out, int64_t *visited)
{
    int rc = check_args(m, n, op, in, out);
    if (rc != OR_OK) return rc;
    int64_t cnt = 0;
    int64_t x[4] = {0, 0, 0, 0};
    if (m == 2) {
        for (x[1] = 0; x[1] <= n; ++x[1])
            for (x[0] = 0; x[0] <= n - x[1]; ++x[0]) {
                apply_one(op, m, n, in, out, x);
                ++cnt;
            }
    } else if (m == 3) {
        for (x[2] = 0; x[2] <= n; ++x[2])
            for (x[1] = 0; x[1] <= n - x[2]; ++x[1])
                for (x[0] = 0; x[0] <= n - x[2] - x[1]; ++x[0]) {
                    apply_one(op, m, n, in, out, x);
                    ++cnt;
                }
    } else {
        for (x[3] = 0; x[3] <= n; ++x[3])
            for (x[2] = 0; x[2] <= n - x[3]; ++x[2])
                for (x[1] = 0; x[1] <= n - x[3] - x[2]; ++x[1])
                    for (x[0] = 0; x[0] <= n - x[3] - x[2] - x[1]; ++x[0]) {
                        apply_one(op, m, n, in, out, x);
                        ++cnt;
                    }
    }
    if (visited) *visited = cnt;
    return OR_OK;
}

/* Same walk, restricted to the slab lo <= x_m < hi of the outermost
 * coordinate (used to time a bounded sample of a large workload). */
int oracle_apply_slab(int m, int64_t n, int op, const void *in, void *out,
                      int64_t lo, int64_t hi, int64_t *visited)
{
    int rc = check_args(m, n, op, in, out);
    if (rc != OR_OK) return rc;
    if (lo < 0) lo = 0;
    if (hi > n + 1) hi = n + 1;
    int64_t cnt = 0;
    int64_t x[4] = {0, 0, 0, 0};
    if (m == 2) {
        for (x[1] = lo; x[1] < hi; ++x[1])
            for (x[0] = 0; x[0] <= n - x[1]; ++x[0]) {
                apply_one(op, m, n, in, out, x);
                ++cnt;
            }
    } else if (m == 3) {
        for (x[2] = lo; x[2] < hi; ++x[2])
            for (x[1] = 0; x[1] <= n - x[2]; ++x[1])
                for (x[0] = 0; x[0] <= n - x[2] - x[1]; ++x[0]) {
                    apply_one(op, m, n, in, out, x);
                    ++cnt;
                }
    } else {
        for (x[3] = lo; x[3] < hi; ++x[3])
            for (x[2] = 0; x[2] <= n - x[3]; ++x[2])
                for (x[1] = 0; x[1] <= n - x[3] - x[2]; ++x[1])
                    for (x[0] = 0; x[0] <= n - x[3] - x[2] - x[1]; ++x[0]) {
                        apply_one(op, m, n, in, out, x);
                        ++cnt;
                    }
    }
    if (visited) *visited = cnt;
    return OR_OK;
}

/* Expected output value at the single element x (which must lie in the
 * simplex), for checking sampled outputs of large runs.  For HITS the value
 * is the increment (1).  in is a full-size box buffer in which at least the
 * cells the definition reads (x, and for CA its neighbours) hold their
 * values.  Returns the value, or -1 if x is outside the simplex. */
int64_t oracle_cell(int m, int64_t n, int op, const void *in, const int64_t *x)
{
    if (m < 2 || m > 4 || !in_simplex(m, n, x)) return -1;
    switch (op) {
    case OR_ACCUM:
        return (int64_t)(uint32_t)(((const uint32_t *)in)[lin_index(m, n, x)] + 1u);
    case OR_HITS:
        return 1;
    case OR_HASH: {
        uint32_t w[4];
        for (int k = 0; k < m; ++k) w[k] = (uint32_t)x[k];
        return (int64_t)oracle_hash32(m, w);
    }
    case OR_CA2:
    case OR_CA3:
        return ca_next(op, m, n, (const uint8_t *)in, x);
    default:
        return 0;
    }
}

/* Expected outputs along one row: x_2..x_m fixed to xhigh[0..m-2], x_1 from
 * 0 to n - (x_2 + ... + x_m).  row_out receives those n+1-sum values
 * (uint32 or uint8 by op).  Returns the row length, or -1 if the row lies
 * outside the simplex or the arguments are bad. */
int64_t oracle_row(int m, int64_t n, int op, const void *in, const int64_t *xhigh, void *row_out)
{
    if (m < 2 || m > 4 || n < 0 || op < OR_MAP || op > OR_CA3 || !row_out) return -1;
    int64_t x[4] = {0, 0, 0, 0}, s = 0;
    for (int k = 1; k < m; ++k) {
        x[k] = xhigh[k - 1];
        if (x[k] < 0) return -1;
        s += x[k];
    }
    if (s > n) return -1;
    const int64_t len = n - s + 1;
    for (x[0] = 0; x[0] < len; ++x[0]) {
        int64_t v = oracle_cell(m, n, op, in, x);
        if (op == OR_CA2 || op == OR_CA3)
            ((uint8_t *)row_out)[x[0]] = (uint8_t)v;
        else
            ((uint32_t *)row_out)[x[0]] = (uint32_t)v;
    }
    return len;
}

/* Number of elements the nested loops visit (must be C(n+m, m)). */
int64_t oracle_count(int m, int64_t n)
{
    int64_t cnt = 0;
    if (oracle_apply(m, n, OR_MAP, NULL, NULL, &cnt) != OR_OK) return -1;
    return cnt;
}


int oracle_edm(int64_t n, const float *pts, double *out, int64_t *visited)
{
    if (n < 0 || pts == NULL || out == NULL) return OR_EINVAL;
    int64_t cnt = 0;
    for (int64_t x2 = 0; x2 <= n; ++x2) {
        for (int64_t x1 = 0; x1 <= n - x2; ++x1) {
            const int64_t i = x1, j = n - x2;
            double s = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double d = (double)pts[3 * i + k] - (double)pts[3 * j + k];
                s += d * d;
            }
            out[x1 + x2 * (n + 1)] = sqrt(s);
            ++cnt;
        }
    }
    if (visited) *visited = cnt;
    return OR_OK;
}
