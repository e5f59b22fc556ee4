/*
 * CPU oracle for augmented-neighborhood-graph search (arXiv 1312.3062).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Everything is single-threaded.  Distances of byte data are exact integers;
 * distances of float data are computed in double precision.  All keys are
 * held as doubles: integer distances below 2^53 compare exactly.
 *
 * Where the paper is silent the following readings are taken (each is
 * repeated at the function that implements it):
 *   - subspace p covers dims [p*d/P, (p+1)*d/P)                       (Sec. 3.2)
 *   - bridge linear id lid = sum_p k_p * K^(P-1-p), subspace 0 most
 *     significant; a bridge's node id is N + lid                         (Sec. 4.1)
 *   - every order is the total order on (distance, id)
 *   - the budget T is strict: at most T distance evaluations, and the
 *     adjacency list being expanded is cut when the T-th one is done     (Alg. 1)
 *   - the main queue holds reference vectors only, at most L of them; when
 *     it is full a better candidate evicts the worst one.  The single
 *     bridge vector that the paper keeps in the queue is held in its own
 *     slot beside it, so it can never be evicted                         (Sec. 4.2)
 *   - k-means: K initial rows from a partial Fisher-Yates shuffle driven
 *     by SplitMix64, ties in assignment go to the smaller codeword index,
 *     byte centroids are rounded half up to integers each iteration, an
 *     empty cluster keeps its centroid                                   (Sec. 4.1)
 *   - bridge graph: each reference keeps its top-t bridges by
 *     (distance, lid); each bridge keeps its b nearest references by
 *     (distance, id), b = 0 meaning all; lists are stored in that order  (Sec. 4.1)
 *   - multi-sequence: each subspace list sorted by (value, codeword index);
 *     tuples come out in (sum, lid) order; a tuple is pushed by its unique
 *     parent, the tuple with its last non-zero rank lowered by one        (Sec. 3.3)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_U8 0
#define ORC_F32 1

/* ------------------------------------------------------------------ */
/* (distance, id) keys                                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    double d;
    int64_t id;
} okey_t;

static int key_less(okey_t a, okey_t b) {
    if (a.d < b.d) return 1;
    if (a.d > b.d) return 0;
    return a.id < b.id;
}

static int key_cmp_qsort(const void* pa, const void* pb) {
    okey_t a = *(const okey_t*)pa, b = *(const okey_t*)pb;
    if (key_less(a, b)) return -1;
    if (key_less(b, a)) return 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Squared Euclidean distance (Sec. 2: NN under the Euclidean metric;  */
/* the squared distance is stored, Sec. 3.2)                           */
/* ------------------------------------------------------------------ */
static double sqdist_u8(const uint8_t* a, const uint8_t* b, int len) {
    int64_t s = 0;
    for (int i = 0; i < len; i++) {
        int64_t t = (int64_t)a[i] - (int64_t)b[i];
        s += t * t;
    }
    return (double)s;
}

static double sqdist_f32(const float* a, const float* b, int len) {
    double s = 0.0;
    for (int i = 0; i < len; i++) {
        double t = (double)a[i] - (double)b[i];
        s += t * t;
    }
    return s;
}

/* distance between row `ra` of A and row `rb` of B, restricted to dims [lo, lo+len) */
static double sqdist_rows(const void* A, int64_t ra, const void* B, int64_t rb, int d, int lo, int len,
                          int dtype) {
    if (dtype == ORC_U8)
        return sqdist_u8((const uint8_t*)A + ra * d + lo, (const uint8_t*)B + rb * d + lo, len);
    return sqdist_f32((const float*)A + ra * d + lo, (const float*)B + rb * d + lo, len);
}

/* ------------------------------------------------------------------ */
/* bfloat16 (precision form of the search for float data).  A bfloat16  */
/* keeps the sign, the 8 exponent bits and the top 7 fraction bits of a */
/* float32.  The value nearest to f is one of the two patterns around   */
/* it: f cut toward zero to 16 bits, or the next one away from zero.     */
/* The nearer one is taken; at equal distance the one whose last kept   */
/* bit is 0.  Inputs are finite.                                        */
/* ------------------------------------------------------------------ */
static double bf16_nearest(float f) {
    uint32_t u, toward, away;
    float ft, fa;
    memcpy(&u, &f, 4);
    toward = u & 0xFFFF0000u;
    away = toward + 0x10000u;
    memcpy(&ft, &toward, 4);
    memcpy(&fa, &away, 4);
    double et = fabs((double)f - (double)ft), ea = fabs((double)fa - (double)f);
    if (et < ea) return (double)ft;
    if (ea < et) return (double)fa;
    return ((toward >> 16) & 1u) ? (double)fa : (double)ft;
}

void orc_bf16_round(const float* x, int64_t n, double* out) {
    for (int64_t i = 0; i < n; i++) out[i] = bf16_nearest(x[i]);
}

/* squared distance from a float query to the bfloat16 copy of a float row */
static double sqdist_f32_bf16(const float* q, const float* x, int len) {
    double s = 0.0;
    for (int i = 0; i < len; i++) {
        double t = (double)q[i] - bf16_nearest(x[i]);
        s += t * t;
    }
    return s;
}

/* ------------------------------------------------------------------ */
/* Bounded set of the best keys: keeps the `cap` smallest keys offered. */
/* Plain unsorted array; every operation scans it.                     */
/* ------------------------------------------------------------------ */
typedef struct {
    okey_t* e;
    int n, cap;
} bset_t;

static int bset_argmax(const bset_t* s) {
    int m = 0;
    for (int i = 1; i < s->n; i++)
        if (key_less(s->e[m], s->e[i])) m = i;
    return m;
}

static int bset_argmin(const bset_t* s) {
    int m = 0;
    for (int i = 1; i < s->n; i++)
        if (key_less(s->e[i], s->e[m])) m = i;
    return m;
}

/* insert if not full; otherwise replace the largest key if the new one is smaller */
static void bset_offer(bset_t* s, okey_t k) {
    if (s->cap <= 0) return;
    if (s->n < s->cap) {
        s->e[s->n++] = k;
        return;
    }
    int m = bset_argmax(s);
    if (key_less(k, s->e[m])) s->e[m] = k;
}

static okey_t bset_pop_min(bset_t* s) {
    int m = bset_argmin(s);
    okey_t k = s->e[m];
    s->e[m] = s->e[s->n - 1];
    s->n--;
    return k;
}

/* ------------------------------------------------------------------ */
/* Exact k nearest neighbours by linear scan (Sec. 1 and Sec. 5.1: the  */
/* ground truth).  exclude[i] >= 0 removes that id from query i's list  */
/* (used for the kNN graph, where a vector is not its own neighbour).   */
/* Output ascending by (distance, id); missing entries get id -1.       */
/* ------------------------------------------------------------------ */
void orc_knn(const void* X, int64_t n, int d, int dtype, const void* Q, int64_t nq, const int64_t* exclude,
             int k, int32_t* out_ids, double* out_d) {
    okey_t* buf = (okey_t*)malloc(sizeof(okey_t) * (size_t)(k > 0 ? k : 1));
    for (int64_t q = 0; q < nq; q++) {
        bset_t s = {buf, 0, k};
        for (int64_t j = 0; j < n; j++) {
            if (exclude && exclude[q] == j) continue;
            okey_t c = {sqdist_rows(Q, q, X, j, d, 0, d, dtype), j};
            bset_offer(&s, c);
        }
        qsort(s.e, (size_t)s.n, sizeof(okey_t), key_cmp_qsort);
        for (int i = 0; i < k; i++) {
            out_ids[q * k + i] = i < s.n ? (int32_t)s.e[i].id : -1;
            out_d[q * k + i] = i < s.n ? s.e[i].d : INFINITY;
        }
    }
    free(buf);
}

/* ------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood 2014), written from its published     */
/* definition: add the golden gamma, then two xor-shift-multiply rounds. */
/* ------------------------------------------------------------------ */
static uint64_t splitmix64_next(uint64_t* state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void orc_splitmix64(uint64_t seed, int64_t count, uint64_t* out) {
    uint64_t s = seed;
    for (int64_t i = 0; i < count; i++) out[i] = splitmix64_next(&s);
}

/* The first K entries of a Fisher-Yates shuffle of [0, n). */
void orc_init_rows(int64_t n, int K, uint64_t seed, int64_t* rows) {
    int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++) perm[i] = i;
    uint64_t s = seed;
    for (int i = 0; i < K; i++) {
        int64_t j = i + (int64_t)(splitmix64_next(&s) % (uint64_t)(n - i));
        int64_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
        rows[i] = perm[i];
    }
    free(perm);
}

/* ------------------------------------------------------------------ */
/* Product-quantisation codebooks (Sec. 3.2 and Sec. 4.1): one k-means  */
/* per subspace.  codebooks is P x K x (d/P), same dtype as X.          */
/* assign (optional, n x P) receives the assignment of the last         */
/* iteration, i.e. the one the final centroids were computed from.      */
/* ------------------------------------------------------------------ */
void orc_kmeans(const void* X, int64_t n, int d, int dtype, int P, int K, int iters, uint64_t seed,
                void* codebooks, int32_t* assign_out) {
    const int ds = d / P;
    int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)K);
    orc_init_rows(n, K, seed, rows);
    int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    double* sum = (double*)malloc(sizeof(double) * (size_t)K * ds);
    int64_t* isum = (int64_t*)malloc(sizeof(int64_t) * (size_t)K * ds);
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)K);
    for (int p = 0; p < P; p++) {
        const int lo = p * ds;
        /* centroid j of subspace p lives at codebooks[(p*K + j)*ds ...] */
        for (int j = 0; j < K; j++)
            for (int e = 0; e < ds; e++) {
                if (dtype == ORC_U8)
                    ((uint8_t*)codebooks)[((int64_t)p * K + j) * ds + e] =
                        ((const uint8_t*)X)[rows[j] * d + lo + e];
                else
                    ((float*)codebooks)[((int64_t)p * K + j) * ds + e] =
                        ((const float*)X)[rows[j] * d + lo + e];
            }
        for (int it = 0; it < iters; it++) {
            /* assignment: nearest centroid, ties to the smaller index */
            for (int64_t i = 0; i < n; i++) {
                int best = 0;
                double bd = 0.0;
                for (int j = 0; j < K; j++) {
                    double dd;
                    if (dtype == ORC_U8)
                        dd = sqdist_u8((const uint8_t*)X + i * d + lo,
                                       (const uint8_t*)codebooks + ((int64_t)p * K + j) * ds, ds);
                    else
                        dd = sqdist_f32((const float*)X + i * d + lo,
                                        (const float*)codebooks + ((int64_t)p * K + j) * ds, ds);
                    if (j == 0 || dd < bd) {
                        bd = dd;
                        best = j;
                    }
                }
                a[i] = best;
            }
            /* update: mean of the members; an empty cluster keeps its centroid */
            memset(cnt, 0, sizeof(int64_t) * (size_t)K);
            memset(isum, 0, sizeof(int64_t) * (size_t)K * ds);
            memset(sum, 0, sizeof(double) * (size_t)K * ds);
            for (int64_t i = 0; i < n; i++) {
                cnt[a[i]]++;
                for (int e = 0; e < ds; e++) {
                    if (dtype == ORC_U8)
                        isum[(int64_t)a[i] * ds + e] += ((const uint8_t*)X)[i * d + lo + e];
                    else
                        sum[(int64_t)a[i] * ds + e] += (double)((const float*)X)[i * d + lo + e];
                }
            }
            for (int j = 0; j < K; j++) {
                if (cnt[j] == 0) continue;
                for (int e = 0; e < ds; e++) {
                    if (dtype == ORC_U8) {
                        /* round half up: floor((2*S + n) / (2*n)) */
                        int64_t v = (2 * isum[(int64_t)j * ds + e] + cnt[j]) / (2 * cnt[j]);
                        ((uint8_t*)codebooks)[((int64_t)p * K + j) * ds + e] = (uint8_t)v;
                    } else {
                        ((float*)codebooks)[((int64_t)p * K + j) * ds + e] =
                            (float)(sum[(int64_t)j * ds + e] / (double)cnt[j]);
                    }
                }
            }
            if (assign_out && it == iters - 1)
                for (int64_t i = 0; i < n; i++) assign_out[i * P + p] = a[i];
        }
        if (assign_out && iters == 0)
            for (int64_t i = 0; i < n; i++) assign_out[i * P + p] = -1;
    }
    free(rows);
    free(a);
    free(sum);
    free(isum);
    free(cnt);
}

/* ------------------------------------------------------------------ */
/* Query preprocessing (Sec. 4.2): squared distances from each query    */
/* subvector to each codeword of its subspace, tab[p*K + j].            */
/* `q` is one vector of the same dtype as the codebooks.                */
/* ------------------------------------------------------------------ */
void orc_tables(const void* q, int d, int dtype, int P, int K, const void* codebooks, double* tab) {
    const int ds = d / P;
    for (int p = 0; p < P; p++)
        for (int j = 0; j < K; j++) {
            if (dtype == ORC_U8)
                tab[p * K + j] = sqdist_u8((const uint8_t*)q + p * ds,
                                           (const uint8_t*)codebooks + ((int64_t)p * K + j) * ds, ds);
            else
                tab[p * K + j] = sqdist_f32((const float*)q + p * ds,
                                            (const float*)codebooks + ((int64_t)p * K + j) * ds, ds);
        }
}

/* Each subspace list sorted ascending by (value, codeword index).      */
/* perm[p*K + r] is the codeword of rank r; sorted[p*K + r] its value.  */
void orc_sort_tables(int P, int K, const double* tab, int32_t* perm, double* sorted) {
    okey_t* tmp = (okey_t*)malloc(sizeof(okey_t) * (size_t)K);
    for (int p = 0; p < P; p++) {
        for (int j = 0; j < K; j++) {
            tmp[j].d = tab[p * K + j];
            tmp[j].id = j;
        }
        qsort(tmp, (size_t)K, sizeof(okey_t), key_cmp_qsort);
        for (int r = 0; r < K; r++) {
            perm[p * K + r] = (int32_t)tmp[r].id;
            sorted[p * K + r] = tmp[r].d;
        }
    }
    free(tmp);
}

/* ------------------------------------------------------------------ */
/* Multi-sequence enumeration (Sec. 3.3; ExtractNextNearestBridgeVector */
/* in Alg. 1).  A min-heap of rank tuples keyed by (sum, lid).           */
/* ------------------------------------------------------------------ */
#define ORC_MAXP 8

typedef struct {
    double sum;
    int64_t lid;
    int32_t r[ORC_MAXP];
} mnode_t;

typedef struct {
    int P, K;
    const int32_t* perm;  /* P x K, codeword of rank r */
    const double* val;    /* P x K, sorted values */
    mnode_t* h;
    int64_t n, cap;
    int64_t emitted, total;
    int64_t max_size;
} mseq_t;

static int mnode_less(const mnode_t* a, const mnode_t* b) {
    if (a->sum < b->sum) return 1;
    if (a->sum > b->sum) return 0;
    return a->lid < b->lid;
}

static void mseq_push(mseq_t* m, const int32_t* r) {
    mnode_t x;
    x.sum = 0.0;
    x.lid = 0;
    for (int p = 0; p < m->P; p++) {
        x.r[p] = r[p];
        x.sum += m->val[p * m->K + r[p]];
        x.lid = x.lid * m->K + m->perm[p * m->K + r[p]];
    }
    if (m->n == m->cap) {
        m->cap = m->cap * 2 + 16;
        m->h = (mnode_t*)realloc(m->h, sizeof(mnode_t) * (size_t)m->cap);
    }
    int64_t i = m->n++;
    m->h[i] = x;
    while (i > 0) { /* sift up */
        int64_t par = (i - 1) / 2;
        if (!mnode_less(&m->h[i], &m->h[par])) break;
        mnode_t t = m->h[i];
        m->h[i] = m->h[par];
        m->h[par] = t;
        i = par;
    }
    if (m->n > m->max_size) m->max_size = m->n;
}

static mnode_t mseq_pop_heap(mseq_t* m) {
    mnode_t top = m->h[0];
    m->h[0] = m->h[--m->n];
    int64_t i = 0;
    for (;;) { /* sift down */
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < m->n && mnode_less(&m->h[l], &m->h[s])) s = l;
        if (r < m->n && mnode_less(&m->h[r], &m->h[s])) s = r;
        if (s == i) break;
        mnode_t t = m->h[i];
        m->h[i] = m->h[s];
        m->h[s] = t;
        i = s;
    }
    return top;
}

static void mseq_init(mseq_t* m, int P, int K, const int32_t* perm, const double* val) {
    m->P = P;
    m->K = K;
    m->perm = perm;
    m->val = val;
    m->h = NULL;
    m->n = m->cap = 0;
    m->emitted = 0;
    m->max_size = 0;
    m->total = 1;
    for (int p = 0; p < P; p++) m->total *= K;
    int32_t zero[ORC_MAXP] = {0};
    mseq_push(m, zero);
}

/* Next bridge in (sum, lid) order.  Returns 0 once all K^P were emitted. */
static int mseq_next(mseq_t* m, int64_t* lid, double* sum) {
    if (m->n == 0) return 0;
    mnode_t x = mseq_pop_heap(m);
    m->emitted++;
    /* unique parent: children raise one rank at or after the last non-zero one */
    int last = 0;
    for (int p = 0; p < m->P; p++)
        if (x.r[p] != 0) last = p;
    for (int b = last; b < m->P; b++) {
        if (x.r[b] + 1 >= m->K) continue;
        int32_t c[ORC_MAXP];
        memcpy(c, x.r, sizeof(int32_t) * (size_t)m->P);
        c[b]++;
        mseq_push(m, c);
    }
    *lid = x.lid;
    *sum = x.sum;
    return 1;
}

static void mseq_free(mseq_t* m) { free(m->h); }

/* The first `count` bridges in increasing distance for the given unsorted */
/* tables; returns how many were emitted (count, or K^P if smaller).        */
int64_t orc_mseq(int P, int K, const double* tab, int64_t count, int64_t* lids, double* sums,
                 int64_t* max_heap) {
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)P * K);
    double* val = (double*)malloc(sizeof(double) * (size_t)P * K);
    orc_sort_tables(P, K, tab, perm, val);
    mseq_t m;
    mseq_init(&m, P, K, perm, val);
    int64_t i = 0;
    while (i < count && mseq_next(&m, &lids[i], &sums[i])) i++;
    if (max_heap) *max_heap = m.max_size;
    mseq_free(&m);
    free(perm);
    free(val);
    return i;
}

/* ------------------------------------------------------------------ */
/* Bridge graph (Sec. 4.1): each reference vector finds its top-t       */
/* bridges by (distance, lid) through its own subspace tables; each      */
/* bridge then keeps its b nearest references by (distance, id), b = 0  */
/* keeping all.  CSR output: off[K^P + 1], ids[E], bdist[E] (distance   */
/* of the reference to that bridge).  Returns E, or -1 if cap is short. */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t lid;
    okey_t k;
} triple_t;

static int triple_cmp(const void* pa, const void* pb) {
    const triple_t* a = (const triple_t*)pa;
    const triple_t* b = (const triple_t*)pb;
    if (a->lid != b->lid) return a->lid < b->lid ? -1 : 1;
    return key_cmp_qsort(&a->k, &b->k);
}

int64_t orc_bridge_graph(const void* X, int64_t n, int d, int dtype, int P, int K, const void* codebooks,
                         int t, int b, uint32_t* off, uint32_t* ids, double* bdist, int64_t cap) {
    int64_t nb = 1;
    for (int p = 0; p < P; p++) nb *= K;
    if (t > nb) t = (int)nb;
    int64_t nt = n * (int64_t)t;
    triple_t* tr = (triple_t*)malloc(sizeof(triple_t) * (size_t)(nt > 0 ? nt : 1));
    double* tab = (double*)malloc(sizeof(double) * (size_t)P * K);
    int64_t* lids = (int64_t*)malloc(sizeof(int64_t) * (size_t)t);
    double* sums = (double*)malloc(sizeof(double) * (size_t)t);
    const size_t esz = dtype == ORC_U8 ? 1 : 4;
    for (int64_t i = 0; i < n; i++) {
        orc_tables((const char*)X + (size_t)i * d * esz, d, dtype, P, K, codebooks, tab);
        int64_t got = orc_mseq(P, K, tab, t, lids, sums, NULL);
        for (int64_t j = 0; j < got; j++) {
            tr[i * t + j].lid = lids[j];
            tr[i * t + j].k.d = sums[j];
            tr[i * t + j].k.id = i;
        }
    }
    /* group by bridge, order each group by (distance, id) */
    qsort(tr, (size_t)nt, sizeof(triple_t), triple_cmp);
    int64_t e = 0, s = 0;
    for (int64_t lid = 0; lid < nb; lid++) {
        off[lid] = (uint32_t)e;
        int64_t kept = 0;
        while (s < nt && tr[s].lid == lid) {
            if (b <= 0 || kept < b) {
                if (e >= cap) {
                    e = -1;
                    goto done;
                }
                ids[e] = (uint32_t)tr[s].k.id;
                if (bdist) bdist[e] = tr[s].k.d;
                e++;
                kept++;
            }
            s++;
        }
    }
    off[nb] = (uint32_t)e;
done:
    free(tr);
    free(tab);
    free(lids);
    free(sums);
    return e;
}

/* ------------------------------------------------------------------ */
/* Alg. 1, ANN search over the augmented neighborhood graph.            */
/*                                                                      */
/* Index: X (n x d), codebooks (P x K x d/P), kNN graph G (n x R, row    */
/* i = Adj[x_i]), bridge graph as CSR (off, ids).  Per query: k results, */
/* budget T.  out_ids / out_d are nq x kmax, ascending by (D, id),      */
/* padded with id -1 and +inf.                                          */
/* trace (optional, nq x tmax): the reference ids in evaluation order.  */
/* stats (optional, nq x 6): evaluations, reference pops, bridge pops,  */
/* bridge-list entries read, adjacency entries read, max heap size.     */
/*                                                                      */
/* Two further forms (orc_search_ex):                                    */
/*  precision 1 (float data only): every distance that drives the       */
/*    search is taken from the bfloat16 copies of the rows (the query    */
/*    stays float); the result set keeps max(k, rerank_k) candidates     */
/*    (rerank_k = 0: k), whose distances are then measured again on the */
/*    float rows and sorted by (D, id); the first k are returned.        */
/*  use_bridges 0: the neighborhood-graph search of Sec. 2.2 without a   */
/*    bridge graph.  The nseeds seed vectors are measured first, in the  */
/*    given order, like the adjacency list of a vertex expanded before   */
/*    anything else; then the main queue is expanded best first.        */
/* ------------------------------------------------------------------ */
void orc_search_ex(const void* X, int64_t n, int d, int dtype, int P, int K, const void* codebooks, int R,
                   const uint32_t* G, const uint32_t* off, const uint32_t* ids, const void* Qv, int64_t nq,
                   const int32_t* ks, const int32_t* Ts, int kmax, int L, int precision, int rerank_k,
                   int use_bridges, const uint32_t* seeds, int nseeds, int32_t* out_ids, double* out_d,
                   int32_t* trace, int tmax, int64_t* stats) {
    const size_t esz = dtype == ORC_U8 ? 1 : 4;
    const int bf16 = dtype == ORC_F32 && precision == 1;
    unsigned char* color = (unsigned char*)calloc((size_t)n, 1); /* 0 = white, 1 = black */
    int64_t* touched = NULL;
    int64_t touched_cap = 0;
    double* tab = (double*)malloc(sizeof(double) * (size_t)P * K);
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)P * K);
    double* val = (double*)malloc(sizeof(double) * (size_t)P * K);
    okey_t* qbuf = (okey_t*)malloc(sizeof(okey_t) * (size_t)(L > 0 ? L : 1));
    int rmax = kmax > rerank_k ? kmax : rerank_k;
    okey_t* rbuf = (okey_t*)malloc(sizeof(okey_t) * (size_t)(rmax > 0 ? rmax : 1));

    for (int64_t qi = 0; qi < nq; qi++) {
        const int k = ks[qi], T = Ts[qi];
        const int rcap = bf16 && rerank_k > k ? rerank_k : k;
        const char* q = (const char*)Qv + (size_t)qi * d * esz;
        int64_t st_eval = 0, st_rpop = 0, st_bpop = 0, st_blist = 0, st_adj = 0;
        if (touched_cap < T) {
            touched_cap = T;
            touched = (int64_t*)realloc(touched, sizeof(int64_t) * (size_t)touched_cap);
        }
        mseq_t ms;
        int have_bridge = 0;
        int64_t blid = 0;
        double bsum = 0.0;
        if (use_bridges) {
            /* query preprocessing: tables and per-subspace sort (Sec. 4.2) */
            orc_tables(q, d, dtype, P, K, codebooks, tab);
            orc_sort_tables(P, K, tab, perm, val);
            mseq_init(&ms, P, K, perm, val);
            have_bridge = mseq_next(&ms, &blid, &bsum); /* nearest bridge vector */
        }

        bset_t Qs = {qbuf, 0, L};
        bset_t Rs = {rbuf, 0, rcap};
        int64_t t = 0;
        /* the seeds of a graph search are measured before anything else */
        const uint32_t* adj = use_bridges ? NULL : seeds;
        int64_t alen = use_bridges ? 0 : nseeds;

        for (;;) {
            for (int64_t a = 0; a < alen; a++) {
                if (t == T) break;
                int64_t x = adj[a];
                if (color[x]) continue;
                color[x] = 1;
                touched[t] = x;
                double dx = bf16 ? sqdist_f32_bf16((const float*)q, (const float*)X + x * d, d)
                                 : sqdist_rows(q, 0, X, x, d, 0, d, dtype);
                okey_t c = {dx, x};
                if (trace && t < tmax) trace[qi * tmax + t] = (int32_t)x;
                t++;
                bset_offer(&Rs, c);
                bset_offer(&Qs, c);
            }
            if (t >= T) break;
            okey_t bkey = {bsum, n + blid};
            if (have_bridge && (Qs.n == 0 || key_less(bkey, Qs.e[bset_argmin(&Qs)]))) {
                /* the top of the main queue is the bridge vector */
                adj = ids + off[blid];
                alen = (int64_t)off[blid + 1] - (int64_t)off[blid];
                st_bpop++;
                st_blist += alen;
                have_bridge = mseq_next(&ms, &blid, &bsum); /* extract the next one */
            } else if (Qs.n > 0) {
                okey_t p = bset_pop_min(&Qs);
                adj = G + p.id * (int64_t)R;
                alen = R;
                st_rpop++;
            } else {
                break; /* queue empty and every bridge vector consumed */
            }
            st_adj += alen;
        }
        if (bf16) /* the kept candidates measured again on the float rows */
            for (int i = 0; i < Rs.n; i++)
                Rs.e[i].d = sqdist_rows(q, 0, X, Rs.e[i].id, d, 0, d, dtype);
        /* results ascending by (D, id), padded */
        qsort(Rs.e, (size_t)Rs.n, sizeof(okey_t), key_cmp_qsort);
        for (int i = 0; i < kmax; i++) {
            int have = i < Rs.n && i < k;
            out_ids[qi * kmax + i] = have ? (int32_t)Rs.e[i].id : -1;
            out_d[qi * kmax + i] = have ? Rs.e[i].d : INFINITY;
        }
        if (trace)
            for (int64_t i = t; i < tmax; i++) trace[qi * tmax + i] = -1;
        st_eval = t;
        if (stats) {
            stats[qi * 6 + 0] = st_eval;
            stats[qi * 6 + 1] = st_rpop;
            stats[qi * 6 + 2] = st_bpop;
            stats[qi * 6 + 3] = st_blist;
            stats[qi * 6 + 4] = st_adj;
            stats[qi * 6 + 5] = use_bridges ? ms.max_size : 0;
        }
        /* every vector white again for the next query */
        for (int64_t i = 0; i < t; i++) color[touched[i]] = 0;
        if (use_bridges) mseq_free(&ms);
    }
    free(color);
    free(touched);
    free(tab);
    free(perm);
    free(val);
    free(qbuf);
    free(rbuf);
}

void orc_search(const void* X, int64_t n, int d, int dtype, int P, int K, const void* codebooks, int R,
                const uint32_t* G, const uint32_t* off, const uint32_t* ids, const void* Qv, int64_t nq,
                const int32_t* ks, const int32_t* Ts, int kmax, int L, int32_t* out_ids, double* out_d,
                int32_t* trace, int tmax, int64_t* stats) {
    orc_search_ex(X, n, d, dtype, P, K, codebooks, R, G, off, ids, Qv, nq, ks, Ts, kmax, L, 0, 0, 1, NULL, 0,
                  out_ids, out_d, trace, tmax, stats);
}

/* ------------------------------------------------------------------ */
/* Graph-D-ADC (Sec. 5, the billion-scale comparison): inverted lists   */
/* whose coarse centres are found by the graph search, each vector      */
/* stored as the product-quantised residual to its list's centre.       */
/* Readings: a residual subvector's code is its nearest codeword (ties  */
/* to the smaller index); a query visits its lists by increasing centre */
/* distance, each list in the stored order, and the candidate list is   */
/* cut at exactly L vectors, inside a list if need be; candidates are   */
/* ranked by the asymmetric distance |q - c - r|^2 (c the list's        */
/* centre, r the codewords of the vector's code concatenated) and then  */
/* by id.                                                               */
/* ------------------------------------------------------------------ */

/* Codes of n residuals (n x d, double) under m subspaces of K float
 * codewords each (codebooks m x K x d/m).  gap (optional, n x m) receives
 * the second-best minus the best squared distance per subvector. */
void orc_pq_encode(const double* Rv, int64_t n, int d, int m, int K, const float* cb, uint8_t* codes,
                   double* gap) {
    const int ds = d / m;
    for (int64_t i = 0; i < n; i++)
        for (int p = 0; p < m; p++) {
            int best = 0;
            double bd = 0.0, second = INFINITY;
            for (int j = 0; j < K; j++) {
                double s = 0.0;
                for (int e = 0; e < ds; e++) {
                    const double t = Rv[i * d + p * ds + e] - (double)cb[((int64_t)p * K + j) * ds + e];
                    s += t * t;
                }
                if (j == 0 || s < bd) {
                    if (j > 0) second = bd;
                    bd = s;
                    best = j;
                } else if (s < second) {
                    second = s;
                }
            }
            codes[i * m + p] = (uint8_t)best;
            if (gap) gap[i * m + p] = second - bd;
        }
}

typedef struct {
    double dist;
    int32_t id;
} orc_cand;

static int orc_cand_cmp(const void* a, const void* b) {
    const orc_cand* x = (const orc_cand*)a;
    const orc_cand* y = (const orc_cand*)b;
    if (x->dist != y->dist) return x->dist < y->dist ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* The re-ranking of Sec. 5 for nq byte queries.  lists (nq x W) names each
 * query's lists in visiting order (-1 entries are skipped); list j holds
 * positions list_off[j] .. list_off[j+1] of list_ids (vector ids) and codes
 * (m bytes per position).  out_ids / out_d are nq x k, ascending by
 * (distance, id), padded with -1 / +infinity.  cand_count (optional, nq)
 * receives the number of candidates ranked. */
void orc_ivf_adc(const uint8_t* Q, int64_t nq, int d, const uint8_t* centres, const uint32_t* list_off,
                 const uint32_t* list_ids, const uint8_t* codes, int m, int K, const float* cb, const int32_t* lists,
                 int W, int64_t L, int k, int32_t* out_ids, double* out_d, int64_t* cand_count) {
    const int ds = d / m;
    int64_t cap = 0;
    orc_cand* cand = NULL;
    for (int64_t qi = 0; qi < nq; qi++) {
        const uint8_t* q = Q + qi * d;
        int64_t c = 0;
        for (int w = 0; w < W && c < L; w++) {
            const int32_t l = lists[qi * W + w];
            if (l < 0) continue;
            for (uint32_t pos = list_off[l]; pos < list_off[l + 1] && c < L; pos++) {
                if (c == cap) {
                    cap = cap ? 2 * cap : 1024;
                    cand = (orc_cand*)realloc(cand, sizeof(orc_cand) * (size_t)cap);
                }
                double s = 0.0;
                for (int p = 0; p < m; p++) {
                    const float* r = cb + ((int64_t)p * K + codes[(int64_t)pos * m + p]) * ds;
                    for (int e = 0; e < ds; e++) {
                        const int j = p * ds + e;
                        const double t = (double)q[j] - (double)centres[(int64_t)l * d + j] - (double)r[e];
                        s += t * t;
                    }
                }
                cand[c].dist = s;
                cand[c].id = (int32_t)list_ids[pos];
                c++;
            }
        }
        if (c > 1) qsort(cand, (size_t)c, sizeof(orc_cand), orc_cand_cmp);
        for (int i = 0; i < k; i++) {
            out_ids[qi * k + i] = i < c ? cand[i].id : -1;
            out_d[qi * k + i] = i < c ? cand[i].dist : INFINITY;
        }
        if (cand_count) cand_count[qi] = c;
    }
    free(cand);
}
