/*
 * ASKIT FP64 reference oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, sequential
 * reading of the method that the HIP library is checked against.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, header or table with the HIP
 * library, and the library never calls it.
 *
 * Method: March, Xiao, Biros, "ASKIT: Approximate Skeletonization
 * Kernel-Independent Treecode in High Dimensions" (arXiv 1410.0260).
 *
 *   or_direct       Eq. (e:problem): u_i = sum_j K(x_i, x_j) w_j, FP64.
 *   or_knn          kappa nearest neighbours by exhaustive search (Sec. 2.2,
 *                   "Computing nearest neighbors"; exact search replaces the
 *                   randomized-tree search, ties broken by point id).
 *   or_rpknn        the paper's approximate search: iterated random
 *                   projection trees, exhaustive search in each leaf.
 *   or_bandwidth    per-source bandwidth h_j for the variable-bandwidth
 *                   Gaussian (Sec. 4, "variable bandwidth").
 *   or_tree         median-split binary tree (Sec. 2.2 tree rule, Fig. tree).
 *   or_node_lists   BuildNeighbors (Alg. 2) with truncation to l by distance
 *                   to the node (Sec. 2.2, "Skeletonization of leaves").
 *   or_sample_rows  sampled rows T_alpha (Eq. e:sk_targets).
 *   or_gauss_matrix K(T_alpha, C_alpha).
 *   or_id           interpolative decomposition by Householder QR with
 *                   column pivoting (Sec. 2.1, Eq. e:id_error).
 *   or_skeletonize  Skeletonize (Alg. 3) bottom-up over the tree.
 *   or_upward       skeleton weights w~ = w(S) + P w(R) (Sec. 2.1 "Far field
 *                   using skeletonization"; Alg. 3 for internal nodes).
 *   or_evaluate     Evaluate (Alg. 4) with neighbour pruning (Eq. e:prune),
 *                   one literal recursion per target.
 *
 * Every floating-point value is FP64 and every distance is the canonical
 * squared distance D(a,b) = sum_k (a_k - b_k)^2 summed in increasing k.
 * The file must be compiled with -ffp-contract=off so that no product is
 * fused into an FMA.
 *
 * Readings of points the paper leaves open (all are restated in the
 * design notes of the repository):
 *   - K(x, y_j) = exp(-D(x, y_j) / (2 h_j^2)), h indexed by the source.
 *   - tree split: centre = mean in a fixed blocked summation order; left
 *     child = the ceil(n/2) smallest projections, ties by point id; each
 *     child keeps its points in increasing point id.
 *   - node-list key = smallest distance from any point of the node to the
 *     neighbour; ties by tree position.
 *   - sampling excludes every point of the node and uses SplitMix64.
 *   - rank k = min(s_max, rows, cols, first t with |R_tt| <= tau' |R_00|),
 *     tau' = max(tau, 64 eps_mach).
 *   - the root is never pruned, so it is never skeletonized.
 *   - "ancestor" in Eq. (e:prune) includes the node itself.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2

typedef struct {
    int32_t lo, hi;     /* points of the node are tree positions [lo, hi) */
    int32_t level;      /* root = 0 */
    int32_t parent;     /* -1 for the root */
    int32_t left, right;/* -1 for a leaf */
    int64_t path;       /* Morton path bits, root = 0, left = 0, right = 1 */
} or_node;

int or_sizeof_node(void) { return (int)sizeof(or_node); }

/* Canonical squared distance: FP64, increasing k, no fused multiply-add. */
static double sqdist(const float *a, const float *b, int d)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = (double)a[k] - (double)b[k];
        s += t * t;
    }
    return s;
}

static double kernel_value(double D, double hj)
{
    return exp(-D / (2.0 * hj * hj));
}

/* ------------------------------------------------------------------ */
/* Eq. (e:problem): direct FP64 kernel sum, targets given by coordinates */
int or_direct(const float *T, int64_t M, const float *X, int64_t N, int d,
              const float *W, int R, const double *hsrc, double h, double *U)
{
    if (M < 0 || N < 1 || d < 1 || R < 1) return OR_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        double *u = U + i * R;
        for (int r = 0; r < R; ++r) u[r] = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            double kij = kernel_value(sqdist(T + i * d, X + j * d, d), hsrc ? hsrc[j] : h);
            for (int r = 0; r < R; ++r) u[r] += kij * (double)W[j * R + r];
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* kappa nearest neighbours, exhaustive: first kappa of {j} sorted by
 * (D(q, x_j), j); with exclude_self, query i skips source j == i.      */
static int nn_less(double d1, int32_t j1, double d2, int32_t j2)
{
    return d1 < d2 || (d1 == d2 && j1 < j2);
}

int or_knn(const float *Q, int64_t M, const float *X, int64_t N, int d, int kappa,
           int exclude_self, int32_t *idx, double *dist)
{
    if (kappa < 1 || N - (exclude_self ? 1 : 0) < kappa || d < 1) return OR_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        int32_t *li = idx + i * kappa;
        double *ld = dist + i * kappa;
        int cnt = 0;
        for (int64_t j = 0; j < N; ++j) {
            if (exclude_self && j == i) continue;
            double D = sqdist(Q + i * d, X + j * d, d);
            if (cnt == kappa && !nn_less(D, (int32_t)j, ld[kappa - 1], li[kappa - 1])) continue;
            int p = cnt < kappa ? cnt++ : kappa - 1;
            while (p > 0 && nn_less(D, (int32_t)j, ld[p - 1], li[p - 1])) {
                ld[p] = ld[p - 1];
                li[p] = li[p - 1];
                --p;
            }
            ld[p] = D;
            li[p] = (int32_t)j;
        }
    }
    return OR_OK;
}

/* Variable bandwidth: h_j = distance from x_j to its b-th neighbour (1-based). */
int or_bandwidth(const double *dist, int64_t N, int kappa, int b, double *h)
{
    if (b < 1 || b > kappa) return OR_EINVAL;
    for (int64_t j = 0; j < N; ++j) h[j] = sqrt(dist[j * kappa + (b - 1)]);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Tree (Sec. 2.2).  Shape depends only on N and m: a node with n > m
 * points has children of ceil(n/2) and floor(n/2) points.  Nodes are
 * numbered breadth first, left before right.                          */
static int64_t count_nodes(int64_t n, int m)
{
    if (n <= m) return 1;
    return 1 + count_nodes((n + 1) / 2, m) + count_nodes(n / 2, m);
}

int64_t or_tree_count(int64_t N, int m)
{
    if (N < 1 || m < 1) return -1;
    return count_nodes(N, m);
}

typedef struct { double p; int32_t id; } proj_t;

static int cmp_proj(const void *a, const void *b)
{
    const proj_t *x = (const proj_t *)a, *y = (const proj_t *)b;
    if (x->p < y->p) return -1;
    if (x->p > y->p) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Centre of the node: per coordinate, blocks of 64 consecutive points (in
 * the node's current order) are summed by pairwise halving (v[t] += v[t+32],
 * then v[t] += v[t+16], ..., v[t] += v[t+1]; absent points count as 0),
 * the block sums are added in block order, and the total is divided by n. */
static void centroid(const float *X, int d, const int32_t *ids, int64_t n, double *c)
{
    double v[64];
    for (int k = 0; k < d; ++k) {
        double acc = 0.0;
        for (int64_t b = 0; b < n; b += 64) {
            for (int t = 0; t < 64; ++t)
                v[t] = (b + t < n) ? (double)X[(int64_t)ids[b + t] * d + k] : 0.0;
            for (int s = 32; s >= 1; s >>= 1)
                for (int t = 0; t < s; ++t) v[t] += v[t + s];
            acc += v[0];
        }
        c[k] = acc / (double)n;
    }
}

static double sqdist_d(const float *a, const double *c, int d)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = (double)a[k] - c[k];
        s += t * t;
    }
    return s;
}

int or_tree(const float *X, int64_t N, int d, int m, or_node *nodes, int64_t nn_cap,
            int32_t *perm)
{
    int64_t nn = or_tree_count(N, m);
    if (nn < 1 || nn > nn_cap || d < 1) return OR_EINVAL;
    double *c = (double *)malloc(sizeof(double) * d);
    proj_t *pr = (proj_t *)malloc(sizeof(proj_t) * (size_t)N);
    if (!c || !pr) { free(c); free(pr); return OR_ENOMEM; }
    for (int64_t i = 0; i < N; ++i) perm[i] = (int32_t)i;
    nodes[0] = (or_node){0, (int32_t)N, 0, -1, -1, -1, 0};
    int64_t next = 1;
    for (int64_t a = 0; a < next; ++a) {          /* breadth-first queue */
        or_node *nd = &nodes[a];
        int64_t lo = nd->lo, n = (int64_t)nd->hi - nd->lo;
        if (n <= m) continue;
        int32_t *ids = perm + lo;
        centroid(X, d, ids, n, c);
        /* x_l = farthest point from the centre; ties to the smaller id */
        int32_t l = -1; double best = -1.0;
        for (int64_t i = 0; i < n; ++i) {
            double D = sqdist_d(X + (int64_t)ids[i] * d, c, d);
            if (D > best || (D == best && ids[i] < l)) { best = D; l = ids[i]; }
        }
        /* x_r = farthest point from x_l; ties to the smaller id */
        int32_t r = -1; best = -1.0;
        for (int64_t i = 0; i < n; ++i) {
            double D = sqdist(X + (int64_t)ids[i] * d, X + (int64_t)l * d, d);
            if (D > best || (D == best && ids[i] < r)) { best = D; r = ids[i]; }
        }
        /* projection on the line (x_l, x_r), relative to x_l */
        const float *xl = X + (int64_t)l * d, *xr = X + (int64_t)r * d;
        for (int64_t i = 0; i < n; ++i) {
            const float *xi = X + (int64_t)ids[i] * d;
            double s = 0.0;
            for (int k = 0; k < d; ++k)
                s += ((double)xi[k] - (double)xl[k]) * ((double)xr[k] - (double)xl[k]);
            pr[i].p = s;
            pr[i].id = ids[i];
        }
        qsort(pr, (size_t)n, sizeof(proj_t), cmp_proj);
        int64_t nl = (n + 1) / 2;
        for (int64_t i = 0; i < n; ++i) ids[i] = pr[i].id;
        qsort(ids, (size_t)nl, sizeof(int32_t), cmp_i32);
        qsort(ids + nl, (size_t)(n - nl), sizeof(int32_t), cmp_i32);
        int64_t L = next++, Rr = next++;
        nodes[L] = (or_node){(int32_t)lo, (int32_t)(lo + nl), nd->level + 1, (int32_t)a, -1, -1,
                             nd->path << 1};
        nodes[Rr] = (or_node){(int32_t)(lo + nl), nd->hi, nd->level + 1, (int32_t)a, -1, -1,
                              (nd->path << 1) | 1};
        nd = &nodes[a];
        nd->left = (int32_t)L;
        nd->right = (int32_t)Rr;
    }
    free(c);
    free(pr);
    return next == nn ? OR_OK : OR_EINVAL;
}

/* ------------------------------------------------------------------ */
/* BuildNeighbors (Alg. 2) with truncation to l nearest (Sec. 2.2).
 * Leaf: N_alpha = (union of N_i, i in alpha) minus alpha, key(j) = min
 * D(x_i, x_j).  Internal: union of the children's stored (truncated)
 * lists minus alpha, key = min of the children's keys.  Sorted by
 * (key, position), truncated to l.  Lists hold tree positions.         */
typedef struct { double key; int32_t pos; } nl_t;

static int cmp_nl_pos(const void *a, const void *b)
{
    const nl_t *x = (const nl_t *)a, *y = (const nl_t *)b;
    if (x->pos != y->pos) return (x->pos > y->pos) - (x->pos < y->pos);
    return (x->key > y->key) - (x->key < y->key);
}

static int cmp_nl_key(const void *a, const void *b)
{
    const nl_t *x = (const nl_t *)a, *y = (const nl_t *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->pos > y->pos) - (x->pos < y->pos);
}

int or_node_lists(const or_node *nodes, int64_t nn, int64_t N, const int32_t *perm,
                  const int32_t *knn_idx, const double *knn_d, int kappa, int ell,
                  int32_t *nl_pos, double *nl_key, int32_t *nl_cnt)
{
    int32_t *iperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!iperm) return OR_ENOMEM;
    for (int64_t i = 0; i < N; ++i) iperm[perm[i]] = (int32_t)i;
    int64_t cap = 2 * (int64_t)ell;
    for (int64_t a = 0; a < nn; ++a) {
        int64_t n = (int64_t)nodes[a].hi - nodes[a].lo;
        if (nodes[a].left < 0 && n * kappa > cap) cap = n * kappa;
    }
    nl_t *e = (nl_t *)malloc(sizeof(nl_t) * (size_t)cap);
    if (!e) { free(iperm); return OR_ENOMEM; }
    for (int64_t a = nn - 1; a >= 0; --a) {     /* children have larger ids */
        const or_node *nd = &nodes[a];
        int64_t cnt = 0;
        if (a == 0) { nl_cnt[a] = 0; continue; }
        if (nd->left < 0) {
            for (int32_t i = nd->lo; i < nd->hi; ++i) {
                int64_t o = perm[i];
                for (int t = 0; t < kappa; ++t) {
                    int32_t pj = iperm[knn_idx[o * kappa + t]];
                    if (pj >= nd->lo && pj < nd->hi) continue;
                    e[cnt].pos = pj;
                    e[cnt].key = knn_d[o * kappa + t];
                    ++cnt;
                }
            }
        } else {
            int32_t ch[2] = {nd->left, nd->right};
            for (int c = 0; c < 2; ++c)
                for (int t = 0; t < nl_cnt[ch[c]]; ++t) {
                    int32_t pj = nl_pos[(int64_t)ch[c] * ell + t];
                    if (pj >= nd->lo && pj < nd->hi) continue;
                    e[cnt].pos = pj;
                    e[cnt].key = nl_key[(int64_t)ch[c] * ell + t];
                    ++cnt;
                }
        }
        qsort(e, (size_t)cnt, sizeof(nl_t), cmp_nl_pos);
        int64_t u = 0;
        for (int64_t t = 0; t < cnt; ++t)
            if (u == 0 || e[u - 1].pos != e[t].pos) e[u++] = e[t];
        qsort(e, (size_t)u, sizeof(nl_t), cmp_nl_key);
        if (u > ell) u = ell;
        for (int64_t t = 0; t < u; ++t) {
            nl_pos[a * ell + t] = e[t].pos;
            nl_key[a * ell + t] = e[t].key;
        }
        nl_cnt[a] = (int32_t)u;
    }
    free(e);
    free(iperm);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Sampled rows (Eq. e:sk_targets): T_alpha = N_alpha followed by
 * r = min(l - |N_alpha|, N - n_alpha - |N_alpha|) positions drawn uniformly
 * without replacement from outside alpha and outside N_alpha.
 *
 * Random stream: the t-th output (t = 0, 1, ...) of SplitMix64 (Steele,
 * Lea, Flood 2014) whose state starts at base = seed XOR (key * golden),
 * key = (level << 48) | path; output(t) = mix(base + (t + 1) * golden).
 * Draw: v = z mod (N - n_alpha); pos = v < lo ? v : v + n_alpha; rejected
 * when pos is in N_alpha or already drawn.  When the pool holds at most 2r
 * positions, the pool is listed in increasing position and the first r
 * entries of a Fisher-Yates shuffle (swap t with t + z_t mod (pool - t))
 * are taken instead.                                                  */
#define SM64_GOLDEN 0x9E3779B97F4A7C15ULL

static uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t or_splitmix64(uint64_t base, uint64_t t)
{
    return sm64_mix(base + (t + 1) * SM64_GOLDEN);
}

static int in_list(const int32_t *a, int64_t n, int32_t v)
{
    for (int64_t i = 0; i < n; ++i)
        if (a[i] == v) return 1;
    return 0;
}

int or_sample_rows(const or_node *nodes, int64_t nn, int64_t N, const int32_t *nl_pos,
                   const int32_t *nl_cnt, int ell, uint64_t seed, int32_t *T, int32_t *T_cnt)
{
    int32_t *pool = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * (int64_t)ell + 4));
    if (!pool) return OR_ENOMEM;
    for (int64_t a = 0; a < nn; ++a) {
        const or_node *nd = &nodes[a];
        int32_t *Ta = T + a * ell;
        if (a == 0) { T_cnt[a] = 0; continue; }
        int64_t na = (int64_t)nd->hi - nd->lo;
        int64_t c = nl_cnt[a];
        for (int64_t t = 0; t < c; ++t) Ta[t] = nl_pos[a * ell + t];
        int64_t npool = N - na - c;
        int64_t r = ell - c < npool ? ell - c : npool;
        uint64_t key = ((uint64_t)nd->level << 48) | (uint64_t)nd->path;
        uint64_t base = seed ^ (key * SM64_GOLDEN);
        if (r > 0 && npool <= 2 * r) {
            int64_t q = 0;
            for (int64_t p = 0; p < N; ++p) {
                if (p >= nd->lo && p < nd->hi) continue;
                if (in_list(Ta, c, (int32_t)p)) continue;
                pool[q++] = (int32_t)p;
            }
            for (int64_t t = 0; t < r; ++t) {
                uint64_t z = or_splitmix64(base, (uint64_t)t);
                int64_t s = t + (int64_t)(z % (uint64_t)(npool - t));
                int32_t tmp = pool[t]; pool[t] = pool[s]; pool[s] = tmp;
                Ta[c + t] = pool[t];
            }
        } else if (r > 0) {
            int64_t got = 0;
            for (uint64_t t = 0; got < r; ++t) {
                uint64_t z = or_splitmix64(base, t);
                int64_t v = (int64_t)(z % (uint64_t)(N - na));
                int32_t pos = (int32_t)(v < nd->lo ? v : v + na);
                if (in_list(Ta, c + got, pos)) continue;
                Ta[c + got++] = pos;
            }
        }
        T_cnt[a] = (int32_t)(c + (r > 0 ? r : 0));
    }
    free(pool);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Approximate neighbours (Sec. 2.2, "Computing nearest neighbors"): greedy
 * search with random projection trees.  One round: build a tree over all
 * points whose nodes split at the median of the projections on a random
 * direction, give every point the other points of its leaf as candidates
 * (exhaustive search), keep its kappa best (D, id) pairs over all rounds so
 * far, discard the tree.
 *
 * Readings: a node with n > leaf points splits into ceil(n/2) (smallest
 * (projection, id)) and floor(n/2), each child in increasing id (the rule of
 * the ASKIT tree, with the random direction in place of (x_l, x_r)); the
 * direction has coordinates +1 or -1 (Achlioptas-type random projection),
 * coordinate k being -1 when bit (k mod 64) of output floor(k / 64) of the
 * SplitMix64 stream with base seed XOR (key * golden) is set, key =
 * ((round + 1) << 53) XOR (level << 48) XOR path; the projection
 * sum_k sign_k x_k is summed in FP64 in increasing k.                    */
typedef struct { int32_t lo, n, level; int64_t path; } rp_node;

static void rp_merge(int32_t *li, double *ld, int kappa, int32_t j, double D)
{
    if (!nn_less(D, j, ld[kappa - 1], li[kappa - 1])) return;
    for (int t = 0; t < kappa; ++t)
        if (li[t] == j) return;               /* already a candidate (same D) */
    int p = kappa - 1;
    while (p > 0 && nn_less(D, j, ld[p - 1], li[p - 1])) {
        ld[p] = ld[p - 1];
        li[p] = li[p - 1];
        --p;
    }
    ld[p] = D;
    li[p] = j;
}

int or_rpknn(const float *X, int64_t N, int d, int kappa, int leaf, int rounds, uint64_t seed,
             int32_t *idx, double *dist)
{
    if (N < 2 || d < 1 || kappa < 1 || kappa >= N || leaf < 2 || rounds < 1) return OR_EINVAL;
    int64_t nn = count_nodes(N, leaf);
    rp_node *nodes = (rp_node *)malloc(sizeof(rp_node) * (size_t)nn);
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    proj_t *pr = (proj_t *)malloc(sizeof(proj_t) * (size_t)N);
    if (!nodes || !ids || !pr) { free(nodes); free(ids); free(pr); return OR_ENOMEM; }
    for (int64_t t = 0; t < N * kappa; ++t) { idx[t] = -1; dist[t] = INFINITY; }
    int rc = OR_OK;
    for (int r = 0; r < rounds && rc == OR_OK; ++r) {
        for (int64_t i = 0; i < N; ++i) ids[i] = (int32_t)i;
        nodes[0] = (rp_node){0, (int32_t)N, 0, 0};
        int64_t next = 1;
        for (int64_t a = 0; a < next; ++a) {      /* breadth first */
            rp_node nd = nodes[a];
            if (nd.n <= leaf) {                    /* leaf: exhaustive search */
                if (nd.n - 1 < kappa) { rc = OR_EINVAL; break; }
                for (int32_t u = 0; u < nd.n; ++u) {
                    int32_t i = ids[nd.lo + u];
                    for (int32_t v = 0; v < nd.n; ++v) {
                        if (v == u) continue;
                        int32_t j = ids[nd.lo + v];
                        rp_merge(idx + (int64_t)i * kappa, dist + (int64_t)i * kappa, kappa, j,
                                 sqdist(X + (int64_t)i * d, X + (int64_t)j * d, d));
                    }
                }
                continue;
            }
            uint64_t key = ((uint64_t)(r + 1) << 53) ^ ((uint64_t)nd.level << 48) ^ (uint64_t)nd.path;
            uint64_t base = seed ^ (key * SM64_GOLDEN);
            for (int32_t u = 0; u < nd.n; ++u) {
                const float *x = X + (int64_t)ids[nd.lo + u] * d;
                double s = 0.0;
                uint64_t z = 0;
                for (int k = 0; k < d; ++k) {
                    if (k % 64 == 0) z = or_splitmix64(base, (uint64_t)(k / 64));
                    if ((z >> (k % 64)) & 1) s -= (double)x[k];
                    else s += (double)x[k];
                }
                pr[u].p = s;
                pr[u].id = ids[nd.lo + u];
            }
            qsort(pr, (size_t)nd.n, sizeof(proj_t), cmp_proj);
            int32_t nl = (nd.n + 1) / 2;
            for (int32_t u = 0; u < nd.n; ++u) ids[nd.lo + u] = pr[u].id;
            qsort(ids + nd.lo, (size_t)nl, sizeof(int32_t), cmp_i32);
            qsort(ids + nd.lo + nl, (size_t)(nd.n - nl), sizeof(int32_t), cmp_i32);
            nodes[next++] = (rp_node){nd.lo, nl, nd.level + 1, nd.path << 1};
            nodes[next++] = (rp_node){nd.lo + nl, nd.n - nl, nd.level + 1, (nd.path << 1) | 1};
        }
    }
    free(nodes);
    free(ids);
    free(pr);
    return rc;
}

/* ------------------------------------------------------------------ */
/* G[t][c] = K(x_rows[t], x_cols[c]) with the column (source) bandwidth.
 * rows/cols are original point ids; G is row-major nr x nc.           */
int or_gauss_matrix(const float *X, int d, const int32_t *rows, int nr, const int32_t *cols,
                    int nc, const double *hsrc, double h, double *G)
{
    for (int t = 0; t < nr; ++t)
        for (int c = 0; c < nc; ++c)
            G[(int64_t)t * nc + c] = kernel_value(
                sqdist(X + (int64_t)rows[t] * d, X + (int64_t)cols[c] * d, d),
                hsrc ? hsrc[cols[c]] : h);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Interpolative decomposition (Sec. 2.1): G Pi = Q R by Householder QR
 * with column pivoting.  Step t pivots on the column of largest residual
 * norm (recomputed from rows t.. of the updated matrix; ties to the lowest
 * current column).  The rank k is the first t with |R_tt| <= tau' |R_00|,
 * tau' = max(tau, 64 eps_mach) (a residual at rounding level counts as
 * zero), k = 0 when R_00 = 0, capped by min(s_max, rows, cols).
 * Skeleton = the first k pivots; P = R11^{-1} R12 (k x (cols-k),
 * row-major), so that G(:, R) ~ G(:, S) P with R = the remaining pivots.
 * The reflector of step t is H = I - beta v v^T with v_t = 1 and
 * v_i = A[i][t] / (A[t][t] - R_tt), beta = (R_tt - A[t][t]) / R_tt,
 * R_tt = -sign(A[t][t]) * norm (sign(0) = +1).
 * piv receives all cols pivots; rdiag receives R_tt for t < k.
 * Margins: the smallest relative gap between the best and second-best
 * squared residual norm over the accepted steps, and the smallest
 * |nrm_t / (tau' nrm_0) - 1| over the rank tests made.                 */
#define OR_ID_TAU_FLOOR (64.0 * 2.220446049250313e-16)

int or_id(const double *G, int rows, int cols, int smax, double tau, int32_t *piv, int32_t *kout,
          double *P, double *rdiag, double *piv_margin, double *rank_margin)
{
    if (rows < 0 || cols < 0 || smax < 0 || !(tau >= 0.0)) return OR_EINVAL;
    double *A = (double *)malloc(sizeof(double) * ((size_t)rows * cols + 1));
    double *v = (double *)malloc(sizeof(double) * ((size_t)rows + 1));
    if (!A || !v) { free(A); free(v); return OR_ENOMEM; }
    memcpy(A, G, sizeof(double) * (size_t)rows * cols);
    for (int c = 0; c < cols; ++c) piv[c] = c;
    double teff = tau > OR_ID_TAU_FLOOR ? tau : OR_ID_TAU_FLOOR;
    int kcap = smax;
    if (rows < kcap) kcap = rows;
    if (cols < kcap) kcap = cols;
    int k = kcap;
    double nrm0 = 0.0, pm = INFINITY, rm = INFINITY;
    for (int t = 0; t < kcap; ++t) {
        int best = -1;
        double bsq = -1.0, ssq = -1.0;
        for (int j = t; j < cols; ++j) {
            double s = 0.0;
            for (int i = t; i < rows; ++i) s += A[(int64_t)i * cols + j] * A[(int64_t)i * cols + j];
            if (s > bsq) { ssq = bsq; bsq = s; best = j; }
            else if (s > ssq) ssq = s;
        }
        if (best < 0) { k = t; break; }              /* non-finite residuals */
        double nrm = sqrt(bsq);
        if (t == 0) {
            nrm0 = nrm;
            if (!(nrm0 > 0.0)) { k = 0; break; }
        } else {
            double g = fabs(nrm / (teff * nrm0) - 1.0);
            if (g < rm) rm = g;
            if (nrm <= teff * nrm0) { k = t; break; }
        }
        if (ssq >= 0.0) {
            double g = (bsq - ssq) / bsq;
            if (g < pm) pm = g;
        }
        if (best != t) {
            for (int i = 0; i < rows; ++i) {
                double tmp = A[(int64_t)i * cols + t];
                A[(int64_t)i * cols + t] = A[(int64_t)i * cols + best];
                A[(int64_t)i * cols + best] = tmp;
            }
            int32_t tp = piv[t]; piv[t] = piv[best]; piv[best] = tp;
        }
        double x0 = A[(int64_t)t * cols + t];
        double rtt = x0 >= 0.0 ? -nrm : nrm;
        double denom = x0 - rtt;
        double beta = (rtt - x0) / rtt;
        v[t] = 1.0;
        for (int i = t + 1; i < rows; ++i) v[i] = A[(int64_t)i * cols + t] / denom;
        for (int j = t + 1; j < cols; ++j) {
            double s = A[(int64_t)t * cols + j];
            for (int i = t + 1; i < rows; ++i) s += v[i] * A[(int64_t)i * cols + j];
            double f = beta * s;
            A[(int64_t)t * cols + j] -= f;
            for (int i = t + 1; i < rows; ++i) A[(int64_t)i * cols + j] -= f * v[i];
        }
        A[(int64_t)t * cols + t] = rtt;
        for (int i = t + 1; i < rows; ++i) A[(int64_t)i * cols + t] = 0.0;
        if (rdiag) rdiag[t] = rtt;
    }
    /* P = R11^{-1} R12 by back substitution, one column of R12 at a time */
    int nr = cols - k;
    for (int c = 0; c < nr; ++c)
        for (int t = k - 1; t >= 0; --t) {
            double s = A[(int64_t)t * cols + k + c];
            for (int q = t + 1; q < k; ++q) s -= A[(int64_t)t * cols + q] * P[(int64_t)q * nr + c];
            P[(int64_t)t * nr + c] = s / A[(int64_t)t * cols + t];
        }
    *kout = k;
    if (piv_margin) *piv_margin = pm;
    if (rank_margin) *rank_margin = rm;
    free(A);
    free(v);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Skeletonize (Alg. 3), bottom-up over every non-root node.  Columns:
 * a leaf uses its points (positions lo..hi-1); an internal node uses
 * S_left followed by S_right.  Rows are the sampled rows T_alpha.
 * Outputs per node a: k[a], S[a*smax + t] (tree positions), the column
 * pivot order colperm[a*ncol_max + c] (indices into the column list),
 * ncols[a], and P in the slot a*smax*ncol_max (row stride ncols-k).    */
int or_skeletonize(const float *X, int64_t N, int d, const int32_t *perm, const or_node *nodes,
                   int64_t nn, const int32_t *T, const int32_t *T_cnt, int ell,
                   const double *hsrc, double h, int smax, double tau, int ncol_max,
                   int32_t *S, int32_t *kout, int32_t *colperm, int32_t *ncols, double *P,
                   double *pmargin, double *rmargin)
{
    (void)N;
    int maxlevel = 0;
    for (int64_t a = 0; a < nn; ++a)
        if (nodes[a].level > maxlevel) maxlevel = nodes[a].level;
    kout[0] = 0;
    ncols[0] = 0;
    pmargin[0] = INFINITY;
    rmargin[0] = INFINITY;
    int err = OR_OK;
    for (int lev = maxlevel; lev >= 1; --lev) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t a = 1; a < nn; ++a) {
            if (nodes[a].level != lev) continue;
            const or_node *nd = &nodes[a];
            int32_t *cpos = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncol_max);
            int32_t *cid = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncol_max);
            int32_t *rid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ell + 1));
            int nc = 0;
            if (nd->left < 0) {
                for (int32_t p = nd->lo; p < nd->hi; ++p) cpos[nc++] = p;
            } else {
                for (int t = 0; t < kout[nd->left]; ++t) cpos[nc++] = S[(int64_t)nd->left * smax + t];
                for (int t = 0; t < kout[nd->right]; ++t) cpos[nc++] = S[(int64_t)nd->right * smax + t];
            }
            int nr = T_cnt[a];
            for (int c = 0; c < nc; ++c) cid[c] = perm[cpos[c]];
            for (int t = 0; t < nr; ++t) rid[t] = perm[T[a * ell + t]];
            double *G = (double *)malloc(sizeof(double) * ((size_t)nr * nc + 1));
            or_gauss_matrix(X, d, rid, nr, cid, nc, hsrc, h, G);
            int32_t k = 0;
            int rc = or_id(G, nr, nc, smax, tau, colperm + a * ncol_max, &k,
                           P + a * (int64_t)smax * ncol_max, NULL, pmargin + a, rmargin + a);
            if (rc != OR_OK) err = rc;
            kout[a] = k;
            ncols[a] = nc;
            for (int t = 0; t < k; ++t) S[a * smax + t] = cpos[colperm[a * ncol_max + t]];
            free(G);
            free(cpos);
            free(cid);
            free(rid);
        }
    }
    return err;
}

/* ------------------------------------------------------------------ */
/* Skeleton weights, bottom-up: Wc = w(X_alpha) (leaf, tree order) or
 * [w~_left; w~_right] (internal); w~_alpha[t] = Wc[piv t] + sum_c
 * P[t][c] Wc[piv k+c].  Wtree is N x R in tree order; Wsk is nn x smax x R. */
int or_upward(const or_node *nodes, int64_t nn, const double *Wtree, int R, int smax,
              const int32_t *kout, const int32_t *colperm, int ncol_max, const int32_t *ncols,
              const double *P, double *Wsk)
{
    double *Wc = (double *)malloc(sizeof(double) * (size_t)ncol_max * R + 1);
    if (!Wc) return OR_ENOMEM;
    for (int64_t a = nn - 1; a >= 1; --a) {
        const or_node *nd = &nodes[a];
        int n = ncols[a], k = kout[a];
        if (nd->left < 0) {
            for (int c = 0; c < n; ++c)
                for (int r = 0; r < R; ++r) Wc[(int64_t)c * R + r] = Wtree[(int64_t)(nd->lo + c) * R + r];
        } else {
            int kl = kout[nd->left];
            for (int c = 0; c < n; ++c) {
                const double *src = c < kl ? Wsk + ((int64_t)nd->left * smax + c) * R
                                           : Wsk + ((int64_t)nd->right * smax + (c - kl)) * R;
                for (int r = 0; r < R; ++r) Wc[(int64_t)c * R + r] = src[r];
            }
        }
        const int32_t *pv = colperm + a * ncol_max;
        const double *Pa = P + a * (int64_t)smax * ncol_max;
        int nrr = n - k;
        for (int t = 0; t < k; ++t)
            for (int r = 0; r < R; ++r) {
                double acc = 0.0;
                for (int c = 0; c < nrr; ++c) acc += Pa[(int64_t)t * nrr + c] * Wc[(int64_t)pv[k + c] * R + r];
                Wsk[((int64_t)a * smax + t) * R + r] = Wc[(int64_t)pv[t] * R + r] + acc;
            }
    }
    free(Wc);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Evaluate (Alg. 4) for targets given by coordinates Y (M x d) and their
 * neighbour positions nb (M x nnb, tree positions, negative = unused).
 * For a target of the point set, nb holds its own position and those of
 * its kappa neighbours; for a new query point, its kappa neighbours.
 * Prune(alpha) holds when no neighbour position lies in [lo, hi).
 * The traversal visits the left child before the right.  Near leaves and
 * pruned nodes are recorded per target (node ids, visit order).
 * Level restriction (Sec. 3, controlling the growth of the error term:
 * start the evaluation at a fixed distance from the leaves): with
 * min_level > 0 a node above that level is never pruned -- the traversal
 * goes on into its children, and a leaf reached above it is summed directly
 * (a near leaf although it holds no neighbour).                         */
typedef struct {
    const float *X; int d; const int32_t *perm; const or_node *nodes;
    const double *hsrc; double h; const float *W; int R;
    const int32_t *S; const int32_t *kout; int smax; const double *Wsk;
    const float *y; const int32_t *nb; int nnb; int minlev;
    double *u, *unear;
    int32_t *near_ids; int32_t near_n; int near_cap;
    int32_t *far_ids; int32_t far_n; int far_cap;
    int overflow;
} ev_ctx;

static int node_has_neighbour(const ev_ctx *e, const or_node *nd)
{
    for (int q = 0; q < e->nnb; ++q) {
        int32_t p = e->nb[q];
        if (p >= nd->lo && p < nd->hi) return 1;
    }
    return 0;
}

static void eval_rec(ev_ctx *e, int32_t a)
{
    const or_node *nd = &e->nodes[a];
    if (!node_has_neighbour(e, nd) && nd->level >= e->minlev) {   /* pruned: skeleton */
        for (int t = 0; t < e->kout[a]; ++t) {
            int32_t o = e->perm[e->S[(int64_t)a * e->smax + t]];
            double kv = kernel_value(sqdist(e->y, e->X + (int64_t)o * e->d, e->d),
                                     e->hsrc ? e->hsrc[o] : e->h);
            for (int r = 0; r < e->R; ++r) e->u[r] += kv * e->Wsk[((int64_t)a * e->smax + t) * e->R + r];
        }
        if (e->far_n < e->far_cap) e->far_ids[e->far_n] = a; else e->overflow = 1;
        e->far_n++;
        return;
    }
    if (nd->left < 0) {                                 /* near leaf: direct */
        for (int32_t p = nd->lo; p < nd->hi; ++p) {
            int32_t o = e->perm[p];
            double kv = kernel_value(sqdist(e->y, e->X + (int64_t)o * e->d, e->d),
                                     e->hsrc ? e->hsrc[o] : e->h);
            for (int r = 0; r < e->R; ++r) {
                double t = kv * (double)e->W[(int64_t)o * e->R + r];
                e->u[r] += t;
                if (e->unear) e->unear[r] += t;
            }
        }
        if (e->near_n < e->near_cap) e->near_ids[e->near_n] = a; else e->overflow = 1;
        e->near_n++;
        return;
    }
    eval_rec(e, nd->left);
    eval_rec(e, nd->right);
}

int or_evaluate(const float *Y, int64_t M, const int32_t *nb, int nnb, const float *X, int d,
                const int32_t *perm, const or_node *nodes, const double *hsrc, double h,
                const float *W, int R, const int32_t *S, const int32_t *kout, int smax,
                const double *Wsk, double *U, double *Unear, int32_t *near_ids, int32_t *near_cnt,
                int near_cap, int32_t *far_ids, int32_t *far_cnt, int far_cap, int min_level)
{
    int overflow = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : overflow)
    for (int64_t i = 0; i < M; ++i) {
        ev_ctx e = {X, d, perm, nodes, hsrc, h, W, R, S, kout, smax, Wsk,
                    Y + i * d, nb + i * nnb, nnb, min_level, U + i * R, Unear ? Unear + i * R : NULL,
                    near_ids ? near_ids + i * near_cap : NULL, 0, near_ids ? near_cap : 0,
                    far_ids ? far_ids + i * far_cap : NULL, 0, far_ids ? far_cap : 0, 0};
        for (int r = 0; r < R; ++r) {
            e.u[r] = 0.0;
            if (e.unear) e.unear[r] = 0.0;
        }
        eval_rec(&e, 0);
        if (near_cnt) near_cnt[i] = e.near_n;
        if (far_cnt) far_cnt[i] = e.far_n;
        if (e.overflow && (near_ids || far_ids)) overflow = 1;
    }
    return overflow ? OR_ENOMEM : OR_OK;
}

/* ------------------------------------------------------------------ */
/* Pruning diagnostic (Table t:prune): nodes visited by the traversal of
 * Alg. 4 for each target, under the neighbour rule of Eq. (e:prune) and under
 * the distance rule the paper compares it with: prune alpha when
 * |x - c_alpha| > R_alpha, c_alpha the centroid of the node's points and
 * R_alpha the largest distance from c_alpha to them.  A call on alpha counts
 * as one visit; a pruned node or a leaf ends the branch, otherwise both
 * children are visited.
 * Readings: the distance rule compares squared distances, D(x, c) > R^2,
 * with R^2 = max D(x_j, c) over the node's points; c is the tree's centroid
 * (the blocked summation of the tree rule over the node's points in
 * increasing id); no extra scaling of R.  Targets are the points
 * themselves; nb holds each target's own position and its neighbours'. */
static int64_t visits_kappa(const or_node *nodes, const int32_t *nb, int nnb)
{
    int32_t stk[128];
    int top = 0;
    int64_t v = 0;
    stk[top++] = 0;
    while (top > 0) {
        const or_node *nd = &nodes[stk[--top]];
        ++v;
        int has = 0;
        for (int q = 0; q < nnb && !has; ++q) has = nb[q] >= nd->lo && nb[q] < nd->hi;
        if (!has || nd->left < 0) continue;
        stk[top++] = nd->right;
        stk[top++] = nd->left;
    }
    return v;
}

static int64_t visits_ball(const or_node *nodes, const float *x, int d, const double *cen, const double *r2)
{
    int32_t stk[128];
    int top = 0;
    int64_t v = 0;
    stk[top++] = 0;
    while (top > 0) {
        int32_t a = stk[--top];
        const or_node *nd = &nodes[a];
        ++v;
        if (sqdist_d(x, cen + (int64_t)a * d, d) > r2[a] || nd->left < 0) continue;
        stk[top++] = nd->right;
        stk[top++] = nd->left;
    }
    return v;
}

int or_prune_visits(const float *X, int64_t N, int d, const int32_t *perm, const or_node *nodes, int64_t nn,
                    const int32_t *nb, int nnb, int32_t *vk, int32_t *vd, double *cen, double *r2)
{
    for (int64_t a = 0; a < nn; ++a) {
        const or_node *nd = &nodes[a];
        int64_t n = (int64_t)nd->hi - nd->lo;
        centroid(X, d, perm + nd->lo, n, cen + a * d);
        double m = 0.0;
        for (int64_t p = nd->lo; p < nd->hi; ++p) {
            double D = sqdist_d(X + (int64_t)perm[p] * d, cen + a * d, d);
            if (D > m) m = D;
        }
        r2[a] = m;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        vk[i] = (int32_t)visits_kappa(nodes, nb + i * nnb, nnb);
        vd[i] = (int32_t)visits_ball(nodes, X + i * d, d, cen, r2);
    }
    return OR_OK;
}
