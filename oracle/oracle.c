/*
 * FP64 CPU oracle for all-mode sparse MTTKRP, dynamic tensor remapping and
 * one CP-ALS sweep (Wijeratne, Kannan, Prasanna: "Dynasor", arXiv 2309.09131).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library: it is written from the
 * paper's definitions, plainly, single-threaded, without SIMD intrinsics,
 * and accumulates in double precision.
 *
 * Every function states the passage it follows.  Parity pins (closed forms,
 * brute force, invariants) live in the tests; none is "parity unpinned".
 *
 * Conventions
 *   idx     N x nnz int32, mode-major: idx[n*nnz + e] is coordinate c_n of
 *           nonzero e (0-based).
 *   vals    nnz doubles (the FP32 tensor values, widened exactly).
 *   factors N pointers, factor n is I_n x R row-major doubles.
 *   Return  0 on success, negative on bad arguments / allocation failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_MODES 8

/* ------------------------------------------------------------------ */
/* 1. Elementwise spMTTKRP (Sec. II-C elementwise update; Eq. 4).       */
/*    M_n(c_n, r) += val * prod_{w != n} A_w(c_w, r), every nonzero in   */
/*    input order.  out_abs (nullable) is the same sum over |val|*|A|,  */
/*    used by the tests as the per-element error scale.                  */
/* ------------------------------------------------------------------ */
int oracle_mttkrp(int N, const int64_t *dims, int64_t nnz, const int32_t *idx,
                  const double *vals, int R, const double *const *factors,
                  int mode, double *out, double *out_abs)
{
    if (N < 2 || N > ORACLE_MAX_MODES || mode < 0 || mode >= N || R < 1)
        return -1;
    int64_t rows = dims[mode];
    memset(out, 0, sizeof(double) * (size_t)rows * R);
    if (out_abs) memset(out_abs, 0, sizeof(double) * (size_t)rows * R);
    double *ell = (double *)malloc(sizeof(double) * R);
    double *ela = (double *)malloc(sizeof(double) * R);
    if (!ell || !ela) { free(ell); free(ela); return -2; }
    for (int64_t e = 0; e < nnz; ++e) {
        for (int r = 0; r < R; ++r) { ell[r] = 1.0; ela[r] = 1.0; }
        for (int w = 0; w < N; ++w) {
            if (w == mode) continue;
            const double *row = factors[w] + (int64_t)idx[(int64_t)w * nnz + e] * R;
            for (int r = 0; r < R; ++r) { ell[r] *= row[r]; ela[r] *= fabs(row[r]); }
        }
        int64_t i = idx[(int64_t)mode * nnz + e];
        double v = vals[e];
        for (int r = 0; r < R; ++r) {
            out[i * R + r] += v * ell[r];
            if (out_abs) out_abs[i * R + r] += fabs(v) * ela[r];
        }
    }
    free(ell); free(ela);
    return 0;
}

/* Same definition restricted to the listed output rows (one by one), so
 * full-size GPU results can be sampled.  out/out_abs are nrows x R. */
int oracle_mttkrp_rows(int N, const int64_t *dims, int64_t nnz,
                       const int32_t *idx, const double *vals, int R,
                       const double *const *factors, int mode, int64_t nrows,
                       const int64_t *rows, double *out, double *out_abs)
{
    if (N < 2 || N > ORACLE_MAX_MODES || mode < 0 || mode >= N || R < 1)
        return -1;
    int64_t I = dims[mode];
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)I);
    if (!slot) return -2;
    for (int64_t i = 0; i < I; ++i) slot[i] = -1;
    for (int64_t k = 0; k < nrows; ++k) {
        if (rows[k] < 0 || rows[k] >= I) { free(slot); return -1; }
        slot[rows[k]] = k;
    }
    memset(out, 0, sizeof(double) * (size_t)nrows * R);
    if (out_abs) memset(out_abs, 0, sizeof(double) * (size_t)nrows * R);
    for (int64_t e = 0; e < nnz; ++e) {
        int64_t k = slot[idx[(int64_t)mode * nnz + e]];
        if (k < 0) continue;
        for (int r = 0; r < R; ++r) {
            double p = vals[e], pa = fabs(vals[e]);
            for (int w = 0; w < N; ++w) {
                if (w == mode) continue;
                double a = factors[w][(int64_t)idx[(int64_t)w * nnz + e] * R + r];
                p *= a; pa *= fabs(a);
            }
            out[k * R + r] += p;
            if (out_abs) out_abs[k * R + r] += pa;
        }
    }
    /* a row listed more than once was summed into the slot of its last
     * listing; every listing gets the row */
    for (int64_t k = 0; k < nrows; ++k) {
        const int64_t k0 = slot[rows[k]];
        if (k0 == k) continue;
        memcpy(out + k * R, out + k0 * R, sizeof(double) * (size_t)R);
        if (out_abs) memcpy(out_abs + k * R, out_abs + k0 * R, sizeof(double) * (size_t)R);
    }
    free(slot);
    return 0;
}

/* ------------------------------------------------------------------ */
/* 2. Layouts.  The tensor starts ordered by mode-0 shards (Sec. III-B); */
/*    while mode n is computed every element is stored into its          */
/*    mode-(n+1) shard (Alg. Dynasor, dynamic remapping store; Sec. IV:  */
/*    the algorithm keeps, per shard of the next mode, the location to   */
/*    fill next).  Within a shard the paper fixes no order; the reading  */
/*    used here is the serial-cursor order, whose fixed point is the     */
/*    cyclic lexicographic order (c_n, c_{n-1}, ..., c_{n+1}, position). */
/* ------------------------------------------------------------------ */
static int g_N;
static int64_t g_nnz;
static const int32_t *g_idx;

static int cmp_l0(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    /* key for L_0: c_0, then c_{N-1}, c_{N-2}, ..., c_1, then position */
    for (int k = 0; k < g_N; ++k) {
        int m = (k == 0) ? 0 : g_N - k;
        int32_t ca = g_idx[(int64_t)m * g_nnz + a], cb = g_idx[(int64_t)m * g_nnz + b];
        if (ca != cb) return ca < cb ? -1 : 1;
    }
    return (a < b) ? -1 : (a > b);
}

/* order[j] = input position of the element at position j of L_0. */
int oracle_canonical_order(int N, int64_t nnz, const int32_t *idx, int64_t *order)
{
    if (N < 2 || N > ORACLE_MAX_MODES || nnz < 0) return -1;
    for (int64_t j = 0; j < nnz; ++j) order[j] = j;
    g_N = N; g_nnz = nnz; g_idx = idx;
    qsort(order, (size_t)nnz, sizeof(int64_t), cmp_l0);
    return 0;
}

/*
 * Serial replay of the remap for one full sweep.
 *   l0        nnz input positions in L_0 order (from oracle_canonical_order)
 *   layouts   (N+1) x nnz: layouts[n*nnz + j] = input position at slot j of
 *             L_n; row N is the layout after the last mode (back to L_0).
 *   perm      N x nnz: perm[n*nnz + i] = destination in L_{n+1} of the
 *             element at slot i of L_n (the per-position remap target).
 *   row_ptr   concatenated per mode, mode n has I_n + 1 entries: exclusive
 *             prefix sum of the number of nonzeros in each mode-n index.
 */
int oracle_remap_replay(int N, const int64_t *dims, int64_t nnz,
                        const int32_t *idx, const int64_t *l0,
                        int64_t *layouts, int64_t *perm, int64_t *row_ptr)
{
    if (N < 2 || N > ORACLE_MAX_MODES || nnz < 0) return -1;
    int64_t off = 0;
    for (int n = 0; n < N; ++n) {
        int64_t *rp = row_ptr + off;
        memset(rp, 0, sizeof(int64_t) * (size_t)(dims[n] + 1));
        for (int64_t e = 0; e < nnz; ++e) {
            int32_t c = idx[(int64_t)n * nnz + e];
            if (c < 0 || c >= dims[n]) return -3;
            rp[c + 1] += 1;
        }
        for (int64_t i = 0; i < dims[n]; ++i) rp[i + 1] += rp[i];
        off += dims[n] + 1;
    }
    memcpy(layouts, l0, sizeof(int64_t) * (size_t)nnz);
    int64_t maxI = 0;
    for (int n = 0; n < N; ++n) if (dims[n] > maxI) maxI = dims[n];
    int64_t *cursor = (int64_t *)malloc(sizeof(int64_t) * (size_t)(maxI + 1));
    if (!cursor) return -2;
    for (int n = 0; n < N; ++n) {
        int nx = (n + 1) % N;
        int64_t rpo = 0;
        for (int k = 0; k < nx; ++k) rpo += dims[k] + 1;
        memcpy(cursor, row_ptr + rpo, sizeof(int64_t) * (size_t)dims[nx]);
        const int64_t *cur = layouts + (int64_t)n * nnz;
        int64_t *next = layouts + (int64_t)(n + 1) * nnz;
        for (int64_t i = 0; i < nnz; ++i) {
            int64_t e = cur[i];
            int32_t c = idx[(int64_t)nx * nnz + e];
            int64_t dst = cursor[c]++;
            perm[(int64_t)n * nnz + i] = dst;
            next[dst] = e;
        }
    }
    free(cursor);
    return 0;
}

/* ------------------------------------------------------------------ */
/* 2b. Locality order (Sec. V-J, preprocessing: Z-Morton ordering of the */
/*    nonzeros).  Reading used for the plan option: each layout L_n keeps */
/*    its output rows contiguous (c_n first) and orders the nonzeros of a */
/*    row by the Morton code of its two leading inputs (c_{n-1}, c_{n-2}), */
/*    then by the remaining inputs c_{n-3}, ..., c_{n+1}, then by input    */
/*    position.  With two modes there is one input and the order is the   */
/*    cyclic lexicographic one.  The remap still moves slot i of L_n to    */
/*    the slot its element takes in L_{n+1}, now computed from the two     */
/*    orders, since L_{n+1} is no longer a stable re-sort of L_n.          */
/* ------------------------------------------------------------------ */

/* Morton code of two 32-bit coordinates: bit k of a goes to bit 2k+1 and
 * bit k of b to bit 2k, so a is the more significant one at every level. */
static uint64_t morton2(uint32_t a, uint32_t b)
{
    uint64_t z = 0;
    for (int k = 0; k < 32; ++k) {
        z |= (uint64_t)((a >> k) & 1u) << (2 * k + 1);
        z |= (uint64_t)((b >> k) & 1u) << (2 * k);
    }
    return z;
}

static int g_mode;

static int32_t coord_of(int m, int64_t e) { return g_idx[(int64_t)m * g_nnz + e]; }

static int cmp_locality(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    const int n = g_mode, N = g_N;
    int32_t ca = coord_of(n, a), cb = coord_of(n, b);
    if (ca != cb) return ca < cb ? -1 : 1;
    int k0 = 1;                                   /* first input not yet compared */
    if (N >= 3) {
        const int m1 = (n + N - 1) % N, m2 = (n + N - 2) % N;
        uint64_t za = morton2((uint32_t)coord_of(m1, a), (uint32_t)coord_of(m2, a));
        uint64_t zb = morton2((uint32_t)coord_of(m1, b), (uint32_t)coord_of(m2, b));
        if (za != zb) return za < zb ? -1 : 1;
        k0 = 3;
    }
    for (int k = k0; k < N; ++k) {                /* c_{n-k}, k = k0 .. N-1 */
        const int m = (n + N - k) % N;
        ca = coord_of(m, a);
        cb = coord_of(m, b);
        if (ca != cb) return ca < cb ? -1 : 1;
    }
    return (a < b) ? -1 : (a > b);
}

/*
 * Layouts and remap targets under the locality order.
 *   layouts  (N+1) x nnz: layouts[n*nnz + j] = input position at slot j of
 *            L_n; row N repeats L_0 (one sweep is a cycle).
 *   perm     N x nnz: perm[n*nnz + i] = slot in L_{n+1} of the element at
 *            slot i of L_n.
 */
int oracle_locality_layouts(int N, const int64_t *dims, int64_t nnz, const int32_t *idx,
                            int64_t *layouts, int64_t *perm)
{
    if (N < 2 || N > ORACLE_MAX_MODES || nnz < 0) return -1;
    for (int n = 0; n < N; ++n)
        for (int64_t e = 0; e < nnz; ++e) {
            int32_t c = idx[(int64_t)n * nnz + e];
            if (c < 0 || c >= dims[n]) return -3;
        }
    g_N = N; g_nnz = nnz; g_idx = idx;
    for (int n = 0; n < N; ++n) {
        int64_t *ord = layouts + (int64_t)n * nnz;
        for (int64_t j = 0; j < nnz; ++j) ord[j] = j;
        g_mode = n;
        qsort(ord, (size_t)nnz, sizeof(int64_t), cmp_locality);
    }
    memcpy(layouts + (int64_t)N * nnz, layouts, sizeof(int64_t) * (size_t)nnz);
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!slot) return -2;
    for (int n = 0; n < N; ++n) {
        const int64_t *cur = layouts + (int64_t)n * nnz;
        const int64_t *next = layouts + (int64_t)(n + 1) * nnz;
        for (int64_t j = 0; j < nnz; ++j) slot[next[j]] = j;     /* element -> slot */
        for (int64_t i = 0; i < nnz; ++i) perm[(int64_t)n * nnz + i] = slot[cur[i]];
    }
    free(slot);
    return 0;
}

/* ------------------------------------------------------------------ */
/* 3. Partitions (Sec. III-A): mode-n indices cut into k_n sets of m_n   */
/*    consecutive indices (last set short: k_n = ceil(I_n / m_n)); the   */
/*    nonzeros incident on set j form super-shard SS_{n,j}; each         */
/*    super-shard is cut into shards of g nonzeros, so mode n has        */
/*    sum_j ceil(|SS_{n,j}| / g) shards.                                 */
/*    row_ptr is the mode's I+1 prefix sum.  Outputs per super-shard:    */
/*    ss_nnz[j], ss_shards[j]; per shard: start, len, super-shard id.    */
/*    *nshards receives the count; shard arrays must hold the bound      */
/*    ceil(nnz/g) + k.                                                   */
/* ------------------------------------------------------------------ */
int oracle_shards(int64_t I, const int64_t *row_ptr, int64_t m, int64_t g,
                  int64_t *ss_nnz, int64_t *ss_shards, int64_t *shard_start,
                  int64_t *shard_len, int64_t *shard_ss, int64_t *nshards)
{
    if (I < 1 || m < 1 || g < 1) return -1;
    int64_t k = (I + m - 1) / m, s = 0;
    for (int64_t j = 0; j < k; ++j) {
        int64_t lo = j * m, hi = (j + 1) * m < I ? (j + 1) * m : I;
        int64_t a = row_ptr[lo], b = row_ptr[hi];
        ss_nnz[j] = b - a;
        ss_shards[j] = (b - a + g - 1) / g;
        for (int64_t q = 0; q < ss_shards[j]; ++q) {
            shard_start[s] = a + q * g;
            shard_len[s] = (a + (q + 1) * g < b ? a + (q + 1) * g : b) - (a + q * g);
            shard_ss[s] = j;
            ++s;
        }
    }
    *nshards = s;
    return 0;
}

/* Super-shard scheduling (Sec. IV-A, Alg. "ss_scheduling"): super-shards
 * sorted by shard count, descending (ties: lower id first), each appended to
 * the bin with the fewest shards so far (ties: lowest bin).  Outputs the bin
 * of each super-shard and the load (shards) of each bin. */
int oracle_lpt(int64_t k, const int64_t *weight, int nu, int32_t *bin_of,
               int64_t *load)
{
    if (k < 0 || nu < 1) return -1;
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
    if (!ord) return -2;
    for (int64_t j = 0; j < k; ++j) ord[j] = j;
    /* insertion sort keeps the plain definition visible; k is small */
    for (int64_t a = 1; a < k; ++a) {
        int64_t x = ord[a], b = a - 1;
        while (b >= 0 && (weight[ord[b]] < weight[x] ||
                          (weight[ord[b]] == weight[x] && ord[b] > x))) {
            ord[b + 1] = ord[b];
            --b;
        }
        ord[b + 1] = x;
    }
    for (int i = 0; i < nu; ++i) load[i] = 0;
    for (int64_t a = 0; a < k; ++a) {
        int best = 0;
        for (int i = 1; i < nu; ++i) if (load[i] < load[best]) best = i;
        bin_of[ord[a]] = best;
        load[best] += weight[ord[a]];
    }
    free(ord);
    return 0;
}

/* ------------------------------------------------------------------ */
/* 4. CP-ALS (Sec. II-B, Alg. "cp-als"), one Gauss-Seidel sweep.         */
/*    The paper's loop assigns each factor from spMTTKRP and normalizes. */
/*    Reading: the standard ALS update from the CPD literature the paper */
/*    cites, A_n = M_n (hadamard_{w!=n} A_w^T A_w)^{-1} via Cholesky,    */
/*    then column 2-norm normalization with weights lambda (a zero       */
/*    column keeps lambda_r = 0 and is left as is).                      */
/* ------------------------------------------------------------------ */
static void gram(const double *A, int64_t I, int R, double *G)
{
    for (int p = 0; p < R; ++p)
        for (int q = 0; q < R; ++q) {
            double s = 0.0;
            for (int64_t i = 0; i < I; ++i) s += A[i * R + p] * A[i * R + q];
            G[p * R + q] = s;
        }
}

/* In-place lower Cholesky of an SPD R x R matrix; returns 0 or -1. */
static int cholesky(double *V, int R)
{
    for (int j = 0; j < R; ++j) {
        double d = V[j * R + j];
        for (int k = 0; k < j; ++k) d -= V[j * R + k] * V[j * R + k];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        V[j * R + j] = d;
        for (int i = j + 1; i < R; ++i) {
            double s = V[i * R + j];
            for (int k = 0; k < j; ++k) s -= V[i * R + k] * V[j * R + k];
            V[i * R + j] = s / d;
        }
        for (int i = 0; i < j; ++i) V[i * R + j] = 0.0;
    }
    return 0;
}

/* Solve x V = b for one row (V = L L^T symmetric): L y = b, L^T x = y. */
static void chol_solve_row(const double *L, int R, const double *b, double *x)
{
    for (int i = 0; i < R; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * R + k] * x[k];
        x[i] = s / L[i * R + i];
    }
    for (int i = R - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k < R; ++k) s -= L[k * R + i] * x[k];
        x[i] = s / L[i * R + i];
    }
}

/*
 * factors:  in/out, N matrices I_n x R (double).
 * lambda:   out, R column weights of the last updated mode.
 * fit:      out (nullable), 1 - ||X - Xhat|| / ||X|| after the sweep.
 * ridge:    out (nullable), number of modes where V needed the ridge
 *           1e-12 * trace(V)/R added before Cholesky succeeded.
 * mode_resid: out (nullable), N entries: ||X - Xhat||^2 after each mode
 *           update (the tests use it for monotonicity on dense tensors).
 */
int oracle_cp_als_sweep(int N, const int64_t *dims, int64_t nnz,
                        const int32_t *idx, const double *vals, int R,
                        double *const *factors, double *lambda, double *fit,
                        int *ridge, double *mode_resid)
{
    if (N < 2 || N > ORACLE_MAX_MODES || R < 1) return -1;
    double *G[ORACLE_MAX_MODES];
    for (int n = 0; n < N; ++n) {
        G[n] = (double *)malloc(sizeof(double) * R * R);
        gram(factors[n], dims[n], R, G[n]);
    }
    double *V = (double *)malloc(sizeof(double) * R * R);
    double *x = (double *)malloc(sizeof(double) * R);
    int64_t maxI = 0;
    for (int n = 0; n < N; ++n) if (dims[n] > maxI) maxI = dims[n];
    double *M = (double *)malloc(sizeof(double) * (size_t)maxI * R);
    double xx = 0.0;
    for (int64_t e = 0; e < nnz; ++e) xx += vals[e] * vals[e];
    if (ridge) *ridge = 0;
    for (int r = 0; r < R; ++r) lambda[r] = 1.0;
    for (int n = 0; n < N; ++n) {
        int64_t I = dims[n];
        oracle_mttkrp(N, dims, nnz, idx, vals, R, (const double *const *)factors,
                      n, M, NULL);
        for (int p = 0; p < R * R; ++p) V[p] = 1.0;
        for (int w = 0; w < N; ++w)
            if (w != n)
                for (int p = 0; p < R * R; ++p) V[p] *= G[w][p];
        double tr = 0.0;
        for (int p = 0; p < R; ++p) tr += V[p * R + p];
        double *Vc = (double *)malloc(sizeof(double) * R * R);
        memcpy(Vc, V, sizeof(double) * R * R);
        if (cholesky(Vc, R) != 0) {
            memcpy(Vc, V, sizeof(double) * R * R);
            for (int p = 0; p < R; ++p) Vc[p * R + p] += 1e-12 * tr / R;
            if (ridge) *ridge += 1;
            if (cholesky(Vc, R) != 0) { free(Vc); return -4; }
        }
        double *A = factors[n];
        for (int64_t i = 0; i < I; ++i) {
            chol_solve_row(Vc, R, M + i * R, x);
            for (int r = 0; r < R; ++r) A[i * R + r] = x[r];
        }
        free(Vc);
        for (int r = 0; r < R; ++r) {
            double s = 0.0;
            for (int64_t i = 0; i < I; ++i) s += A[i * R + r] * A[i * R + r];
            lambda[r] = sqrt(s);
            if (lambda[r] > 0.0)
                for (int64_t i = 0; i < I; ++i) A[i * R + r] /= lambda[r];
        }
        gram(A, I, R, G[n]);
        if (mode_resid || (fit && n == N - 1)) {
            /* <X, Xhat> = sum_r lambda_r sum_i M_n(i,r) A_n(i,r);
             * ||Xhat||^2 = lambda^T (hadamard_w G_w) lambda             */
            double inner = 0.0, nrm = 0.0;
            for (int r = 0; r < R; ++r) {
                double s = 0.0;
                for (int64_t i = 0; i < I; ++i) s += M[i * R + r] * A[i * R + r];
                inner += lambda[r] * s;
            }
            for (int p = 0; p < R; ++p)
                for (int q = 0; q < R; ++q) {
                    double h = 1.0;
                    for (int w = 0; w < N; ++w) h *= G[w][p * R + q];
                    nrm += lambda[p] * lambda[q] * h;
                }
            double res2 = xx - 2.0 * inner + nrm;
            if (mode_resid) mode_resid[n] = res2;
            if (fit && n == N - 1)
                *fit = 1.0 - sqrt(res2 > 0.0 ? res2 : 0.0) / sqrt(xx);
        }
    }
    for (int n = 0; n < N; ++n) free(G[n]);
    free(V); free(x); free(M);
    return 0;
}

/* ------------------------------------------------------------------ */
/* 5. Sampled CP reconstruction loss and its gradient.                  */
/*    Model (Eq. 1, CP approximation): m_e = sum_r prod_n A_n(c_n, r).   */
/*    L = sum_e (x_e - m_e)^2 ; no 1/2, no mean, no weights.             */
/*    dL/dA_k(i, r) = -2 sum_{e: c_k = i} rho_e prod_{n != k} A_n(c_n,r) */
/*    with rho_e = x_e - m_e.  grads (nullable) are N matrices I_n x R.  */
/* ------------------------------------------------------------------ */
int oracle_cp_loss_grad(int N, const int64_t *dims, int64_t nnz,
                        const int32_t *idx, const double *vals, int R,
                        const double *const *factors, double *loss,
                        double *const *grads)
{
    if (N < 2 || N > ORACLE_MAX_MODES || R < 1) return -1;
    if (grads)
        for (int k = 0; k < N; ++k)
            memset(grads[k], 0, sizeof(double) * (size_t)dims[k] * R);
    double L = 0.0;
    for (int64_t e = 0; e < nnz; ++e) {
        double m = 0.0;
        for (int r = 0; r < R; ++r) {
            double p = 1.0;
            for (int n = 0; n < N; ++n)
                p *= factors[n][(int64_t)idx[(int64_t)n * nnz + e] * R + r];
            m += p;
        }
        double rho = vals[e] - m;
        L += rho * rho;
        if (!grads) continue;
        for (int k = 0; k < N; ++k) {
            int64_t i = idx[(int64_t)k * nnz + e];
            for (int r = 0; r < R; ++r) {
                double p = 1.0;
                for (int n = 0; n < N; ++n)
                    if (n != k)
                        p *= factors[n][(int64_t)idx[(int64_t)n * nnz + e] * R + r];
                grads[k][i * R + r] += -2.0 * rho * p;
            }
        }
    }
    if (loss) *loss = L;
    return 0;
}
