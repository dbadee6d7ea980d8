/*
 * CPU oracle for batched B+-tree operations.  TEST INFRASTRUCTURE ONLY:
 * tests, the smoke check and the CPU-baseline leg of the benchmark load it;
 * the GPU library never does, and it shares no code, header or table with
 * the GPU library.
 *
 * Three parts, all plain and single-purpose:
 *
 *  O2  sorted-array reference.  The state S is a sorted array of distinct
 *      keys with their values.  lookup(S,k) is a binary search; an insert
 *      batch is the sequential application of its (key, value) pairs in
 *      batch order, computed as stable sort + last-writer-per-key + merge;
 *      a delete batch removes its keys in batch order (a binary search per
 *      key marks the hits, one pass keeps the rest); range(S, lo, hi, max) is the ascending slice lo <= key <= hi cut to
 *      its first max pairs.  A search that misses reports the paper's -1
 *      (all ones at the key width) together with found = 0 (Section IV-D).
 *
 *  O3  pointer B+-tree in the textbook form of Section III: order m (at
 *      most m children per inner node, at least m/2 for a non-root inner
 *      node), data only in the leaves, leaves chained left to right.  Inner
 *      entry i holds the largest key of child i's subtree, and a search key
 *      goes to the first child whose entry is >= the key (the routing
 *      comparison of Section IV-E).  Inserts go one key
 *      at a time with the classic split; bulk load fills leaves evenly.  It
 *      is the timed CPU baseline (the paper times a CPU B+-tree library,
 *      Section V-F), with lookup batches split evenly over threads.
 *
 *  O4  invariant checker over the flat export format of a tree (header,
 *      inner records, leaf records; the format is documented in gtree.h and
 *      restated below).  It checks sorted leaves, equal leaf depth, fill,
 *      separator bounds, the leaf chain, reachability and the padding rules,
 *      and returns the in-order (key, value) sequence so the caller can
 *      compare it with O2.
 *
 * All keys and values are handled as uint64_t; 32-bit trees are widened by
 * the caller.  `width` (32 or 64) only decides the all-ones miss value and
 * the largest key.
 */
#define _POSIX_C_SOURCE 200809L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <time.h>

typedef uint64_t u64;
typedef uint32_t u32;

static u64 ones(int width) { return width == 32 ? 0xFFFFFFFFull : ~0ull; }

/* ------------------------------------------------------------------ O2 -- */

/* index of the first element >= k in a[0..n) */
static u64 lower_bound(const u64* a, u64 n, u64 k) {
    u64 lo = 0, hi = n;
    while (lo < hi) {
        u64 mid = lo + (hi - lo) / 2;
        if (a[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

void ora_lookup(const u64* keys, const u64* vals, u64 n, const u64* q, u64 B, int width,
                u64* vout, uint8_t* fout) {
    for (u64 i = 0; i < B; i++) {
        u64 p = lower_bound(keys, n, q[i]);
        if (p < n && keys[p] == q[i]) { vout[i] = vals[p]; fout[i] = 1; }
        else { vout[i] = ones(width); fout[i] = 0; }
    }
}

/* (key, batch index) pairs ordered by key then index: a stable key sort. */
typedef struct { u64 key; u64 idx; } kidx;
static int cmp_kidx(const void* a, const void* b) {
    const kidx* x = a; const kidx* y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/*
 * Apply the batch (k[i], v[i]), i = 0..B-1, to S in batch order.
 * status[i] = 0 (INSERTED) if k[i] was absent from S and from k[0..i-1],
 * else 1 (UPDATED).  The final value of a key is that of its last occurrence.
 * out_keys/out_vals need room for n + B entries.  Returns the new size.
 */
u64 ora_insert(const u64* keys, const u64* vals, u64 n, const u64* k, const u64* v, u64 B,
               u64* out_keys, u64* out_vals, uint8_t* status) {
    kidx* s = malloc(sizeof(kidx) * (B ? B : 1));
    for (u64 i = 0; i < B; i++) { s[i].key = k[i]; s[i].idx = i; }
    qsort(s, B, sizeof(kidx), cmp_kidx);
    /* unique batch keys with their final value */
    u64* uk = malloc(sizeof(u64) * (B ? B : 1));
    u64* uv = malloc(sizeof(u64) * (B ? B : 1));
    u64 nu = 0;
    for (u64 i = 0; i < B;) {
        u64 j = i;
        while (j + 1 < B && s[j + 1].key == s[i].key) j++;
        u64 p = lower_bound(keys, n, s[i].key);
        int present = (p < n && keys[p] == s[i].key);
        status[s[i].idx] = present ? 1 : 0;
        for (u64 t = i + 1; t <= j; t++) status[s[t].idx] = 1;
        uk[nu] = s[i].key; uv[nu] = v[s[j].idx]; nu++;
        i = j + 1;
    }
    /* merge S with the unique batch keys; batch value wins on equal keys */
    u64 a = 0, b = 0, o = 0;
    while (a < n || b < nu) {
        if (b >= nu || (a < n && keys[a] < uk[b])) { out_keys[o] = keys[a]; out_vals[o] = vals[a]; a++; }
        else if (a >= n || uk[b] < keys[a]) { out_keys[o] = uk[b]; out_vals[o] = uv[b]; b++; }
        else { out_keys[o] = uk[b]; out_vals[o] = uv[b]; a++; b++; }
        o++;
    }
    free(s); free(uk); free(uv);
    return o;
}

/*
 * Delete the keys k[i], i = 0..B-1, from S in batch order: sequential
 * deletion on the state alone (the paper defines no delete; the tree side
 * keeps the half-full rule of Section III).  status[i] = 1 (DELETED) if
 * k[i] was in S and not earlier in the batch, else 0 (ABSENT).  Each key of
 * S is kept unless some k[i] equals it: a binary search of S per batch key
 * marks the hits, then one pass copies the unmarked pairs.  out_keys and
 * out_vals need room for n entries.  Returns the new size.
 */
u64 ora_delete(const u64* keys, const u64* vals, u64 n, const u64* k, u64 B,
               u64* out_keys, u64* out_vals, uint8_t* status) {
    uint8_t* gone = calloc(n ? n : 1, 1);
    for (u64 i = 0; i < B; i++) {
        u64 p = lower_bound(keys, n, k[i]);
        int present = p < n && keys[p] == k[i] && !gone[p];
        status[i] = present ? 1 : 0;
        if (present) gone[p] = 1;
    }
    u64 o = 0;
    for (u64 a = 0; a < n; a++) {
        if (gone[a]) continue;
        out_keys[o] = keys[a]; out_vals[o] = vals[a]; o++;
    }
    free(gone);
    return o;
}

/*
 * range(S, lo[i], hi[i], max[i]) written at out[off[i] ...]; count[i] pairs.
 * An empty interval (lo > hi) yields no pairs.
 */
void ora_range(const u64* keys, const u64* vals, u64 n, const u64* lo, const u64* hi,
               const u32* maxc, const u64* off, u64 B, u64* out_keys, u64* out_vals, u32* count) {
    for (u64 i = 0; i < B; i++) {
        u64 p = lower_bound(keys, n, lo[i]);
        u32 c = 0;
        while (p < n && keys[p] <= hi[i] && lo[i] <= hi[i] && c < maxc[i]) {
            out_keys[off[i] + c] = keys[p]; out_vals[off[i] + c] = vals[p];
            c++; p++;
        }
        count[i] = c;
    }
}

/* ------------------------------------------------------ O2, byte keys -- */

/*
 * Keys of kb bytes (the paper's 32-byte search keys, Section IV-C).  Two
 * keys compare as byte strings: the first byte in which they differ decides,
 * bytes taken as unsigned and byte 0 first.  That is the order the paper's
 * 32 per-byte comparators reach once its cascading priority rule has picked
 * the most significant byte that is not equal (Section IV-E), i.e. memcmp.
 * Values are 8 bytes, the paper's data entries (Section IV-B).  Keys are
 * packed kb bytes apart; the oracle keeps them sorted and distinct.
 */

/* ascending order of n packed keys: idx receives a permutation of 0..n-1,
 * ties kept in input order (a plain top-down merge sort) */
static void msort_idx(const uint8_t* keys, int kb, u64* idx, u64* tmp, u64 lo, u64 hi) {
    if (hi - lo < 2) return;
    u64 mid = lo + (hi - lo) / 2;
    msort_idx(keys, kb, idx, tmp, lo, mid);
    msort_idx(keys, kb, idx, tmp, mid, hi);
    u64 a = lo, b = mid, o = lo;
    while (a < mid || b < hi) {
        if (b >= hi || (a < mid && memcmp(keys + idx[a] * kb, keys + idx[b] * kb, (size_t)kb) <= 0))
            tmp[o++] = idx[a++];
        else
            tmp[o++] = idx[b++];
    }
    memcpy(idx + lo, tmp + lo, (hi - lo) * sizeof(u64));
}

/*
 * Sort n (key, value) pairs by key into out_keys/out_vals.  Returns 0, or 1
 * when two keys are equal (a tree holds each key once; the output is then
 * sorted but not distinct).
 */
int orb_sort(const uint8_t* keys, const u64* vals, u64 n, int kb, uint8_t* out_keys, u64* out_vals) {
    u64* idx = malloc(sizeof(u64) * (n ? n : 1));
    u64* tmp = malloc(sizeof(u64) * (n ? n : 1));
    for (u64 i = 0; i < n; i++) idx[i] = i;
    msort_idx(keys, kb, idx, tmp, 0, n);
    int dup = 0;
    for (u64 i = 0; i < n; i++) {
        memcpy(out_keys + i * kb, keys + idx[i] * kb, (size_t)kb);
        out_vals[i] = vals[idx[i]];
        if (i && memcmp(out_keys + (i - 1) * kb, out_keys + i * kb, (size_t)kb) == 0) dup = 1;
    }
    free(idx); free(tmp);
    return dup;
}

/* index of the first of the n sorted keys that is >= k */
static u64 lower_bound_b(const uint8_t* keys, u64 n, int kb, const uint8_t* k) {
    u64 lo = 0, hi = n;
    while (lo < hi) {
        u64 mid = lo + (hi - lo) / 2;
        if (memcmp(keys + mid * kb, k, (size_t)kb) < 0) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* lookup: the value of q[i] if present, else all ones, and found 1 / 0 */
void orb_lookup(const uint8_t* keys, const u64* vals, u64 n, int kb, const uint8_t* q, u64 B,
                u64* vout, uint8_t* fout) {
    for (u64 i = 0; i < B; i++) {
        const uint8_t* k = q + i * kb;
        u64 p = lower_bound_b(keys, n, kb, k);
        if (p < n && memcmp(keys + p * kb, k, (size_t)kb) == 0) { vout[i] = vals[p]; fout[i] = 1; }
        else { vout[i] = ~0ull; fout[i] = 0; }
    }
}

/* range: the pairs with lo[i] <= key <= hi[i], ascending, the first maxc[i]
 * of them, written from position off[i]; count[i] = how many */
void orb_range(const uint8_t* keys, const u64* vals, u64 n, int kb, const uint8_t* lo, const uint8_t* hi,
               const u32* maxc, const u64* off, u64 B, uint8_t* out_keys, u64* out_vals, u32* count) {
    for (u64 i = 0; i < B; i++) {
        const uint8_t* l = lo + i * kb;
        const uint8_t* h = hi + i * kb;
        u64 p = lower_bound_b(keys, n, kb, l);
        u32 c = 0;
        if (memcmp(l, h, (size_t)kb) <= 0)
            while (p < n && memcmp(keys + p * kb, h, (size_t)kb) <= 0 && c < maxc[i]) {
                memcpy(out_keys + (off[i] + c) * kb, keys + p * kb, (size_t)kb);
                out_vals[off[i] + c] = vals[p];
                c++; p++;
            }
        count[i] = c;
    }
}

/* ------------------------------------------------------------------ O3 -- */

#define MAXF 64 /* largest order supported */

typedef struct bnode {
    int leaf;
    int n;                        /* leaf: keys held; inner: children */
    u64* key;                     /* leaf: keys; inner: key[i] = max of child i (i < n-1) */
    u64* val;                     /* leaf only */
    struct bnode** child;         /* inner only */
    struct bnode* next;           /* leaf chain */
    u64 tag;                      /* scratch id used by export */
} bnode;

typedef struct {
    int fanout, cap, width;
    bnode* root;
    int height;                   /* levels, leaves included */
    u64 n_keys;
    u64 n_inner, n_leaves;
} bptree;

/* one allocation per node: header, then key[] and val[] or child[], each
   with one spare slot for the transient overflow before a split */
static bnode* new_node(bptree* t, int leaf) {
    int slots = (leaf ? t->cap : t->fanout) + 1;
    bnode* x = calloc(1, sizeof(bnode) + (size_t)slots * 16);
    x->key = (u64*)(x + 1);
    if (leaf) x->val = x->key + slots; else x->child = (bnode**)(x->key + slots);
    x->leaf = leaf;
    if (leaf) t->n_leaves++; else t->n_inner++;
    return x;
}

static void free_rec(bnode* x) {
    if (!x) return;
    if (!x->leaf) for (int i = 0; i < x->n; i++) free_rec(x->child[i]);
    free(x);
}

bptree* bpt_create(int fanout, int cap, int width) {
    if (fanout < 4 || fanout > MAXF || cap < 2 || cap > MAXF) return NULL;
    bptree* t = calloc(1, sizeof(bptree));
    t->fanout = fanout; t->cap = cap; t->width = width;
    t->root = new_node(t, 1);
    t->height = 1;
    return t;
}

void bpt_free(bptree* t) { if (t) { free_rec(t->root); free(t); } }

/* child slot for key k: first i < n-1 with k <= key[i], else n-1 */
static int route(const bnode* x, u64 k) {
    int i = 0;
    while (i < x->n - 1 && x->key[i] < k) i++;
    return i;
}

/* largest key in a subtree (rightmost leaf's last key) */
static u64 subtree_max(const bnode* x) {
    while (!x->leaf) x = x->child[x->n - 1];
    return x->key[x->n - 1];
}

/*
 * Number of nodes a level of `items` entries is packed into, at most `cap`
 * per node after the fill factor, at least cap/2 per node when there are two
 * or more nodes, one node for a small level.
 */
static u64 pack_count(u64 items, int cap, double fill) {
    u64 per = (u64)(cap * fill);
    if (per < 1) per = 1;
    u64 a = (items + per - 1) / per;
    u64 b = items / (u64)((cap + 1) / 2);
    u64 c = a < b ? a : b;
    return c < 1 ? 1 : c;
}

/* keys must be strictly ascending; returns 0 on success, -1 otherwise */
int bpt_bulk_load(bptree* t, const u64* keys, const u64* vals, u64 n, double fill) {
    for (u64 i = 1; i < n; i++) if (keys[i - 1] >= keys[i]) return -1;
    free_rec(t->root);
    t->n_inner = t->n_leaves = 0;
    t->n_keys = n;
    if (n == 0) { t->root = new_node(t, 1); t->height = 1; return 0; }
    u64 L = pack_count(n, t->cap, fill);
    bnode** level = malloc(sizeof(bnode*) * L);
    for (u64 j = 0; j < L; j++) {
        u64 b = j * n / L, e = (j + 1) * n / L;
        bnode* x = new_node(t, 1);
        x->n = (int)(e - b);
        for (u64 i = b; i < e; i++) { x->key[i - b] = keys[i]; x->val[i - b] = vals[i]; }
        level[j] = x;
        if (j) level[j - 1]->next = x;
    }
    u64 cnt = L;
    int h = 1;
    while (cnt > 1) {
        u64 P = pack_count(cnt, t->fanout, fill);
        bnode** up = malloc(sizeof(bnode*) * P);
        for (u64 j = 0; j < P; j++) {
            u64 b = j * cnt / P, e = (j + 1) * cnt / P;
            bnode* x = new_node(t, 0);
            x->n = (int)(e - b);
            for (u64 i = b; i < e; i++) {
                x->child[i - b] = level[i];
                if (i + 1 < e) x->key[i - b] = subtree_max(level[i]);
            }
            up[j] = x;
        }
        free(level);
        level = up; cnt = P; h++;
    }
    t->root = level[0];
    t->height = h;
    free(level);
    return 0;
}

/*
 * Insert into the subtree x.  If x overflows it is split in two; the new
 * right sibling is returned through *right and x's new largest key through
 * *lmax.  Returns 1 if the key was present (value overwritten), else 0.
 */
static int ins_rec(bptree* t, bnode* x, u64 k, u64 v, bnode** right, u64* lmax) {
    *right = NULL;
    if (x->leaf) {
        int p = 0;
        while (p < x->n && x->key[p] < k) p++;
        if (p < x->n && x->key[p] == k) { x->val[p] = v; return 1; }
        for (int i = x->n; i > p; i--) { x->key[i] = x->key[i - 1]; x->val[i] = x->val[i - 1]; }
        x->key[p] = k; x->val[p] = v; x->n++;
        t->n_keys++;
        if (x->n > t->cap) {
            bnode* r = new_node(t, 1);
            int left = (x->n + 1) / 2;
            r->n = x->n - left;
            for (int i = 0; i < r->n; i++) { r->key[i] = x->key[left + i]; r->val[i] = x->val[left + i]; }
            x->n = left;
            r->next = x->next; x->next = r;
            *right = r; *lmax = x->key[left - 1];
        }
        return 0;
    }
    int c = route(x, k);
    bnode* cr; u64 cm;
    int upd = ins_rec(t, x->child[c], k, v, &cr, &cm);
    if (cr) {
        /* child c became (child c, cr): entry c's bound becomes cm, cr takes
           the old bound of entry c */
        for (int i = x->n; i > c + 1; i--) { x->child[i] = x->child[i - 1]; x->key[i] = x->key[i - 1]; }
        x->key[c + 1] = x->key[c];
        x->child[c + 1] = cr;
        x->key[c] = cm;
        x->n++;
        if (x->n > t->fanout) {
            bnode* r = new_node(t, 0);
            int left = (x->n + 1) / 2;
            r->n = x->n - left;
            for (int i = 0; i < r->n; i++) { r->child[i] = x->child[left + i]; r->key[i] = x->key[left + i]; }
            x->n = left;
            *right = r; *lmax = x->key[left - 1];
        }
    }
    return upd;
}

int bpt_insert(bptree* t, u64 k, u64 v) {
    bnode* r; u64 m;
    int upd = ins_rec(t, t->root, k, v, &r, &m);
    if (r) {
        bnode* nr = new_node(t, 0);
        nr->n = 2;
        nr->child[0] = t->root; nr->child[1] = r;
        nr->key[0] = m;
        t->root = nr;
        t->height++;
    }
    return upd;
}

/* sequential application of a batch; status as in ora_insert */
void bpt_insert_batch(bptree* t, const u64* k, const u64* v, u64 B, uint8_t* status) {
    for (u64 i = 0; i < B; i++) status[i] = (uint8_t)bpt_insert(t, k[i], v[i]);
}

static int find1(const bptree* t, u64 k, u64* out) {
    const bnode* x = t->root;
    while (!x->leaf) x = x->child[route(x, k)];
    int lo = 0, hi = x->n;
    while (lo < hi) { int m = (lo + hi) / 2; if (x->key[m] < k) lo = m + 1; else hi = m; }
    if (lo < x->n && x->key[lo] == k) { *out = x->val[lo]; return 1; }
    return 0;
}

typedef struct { const bptree* t; const u64* q; u64 b, e; u64* vout; uint8_t* fout; } lk_job;

static void* lk_worker(void* p) {
    lk_job* j = p;
    u64 miss = ones(j->t->width);
    for (u64 i = j->b; i < j->e; i++) {
        u64 v;
        if (find1(j->t, j->q[i], &v)) { j->vout[i] = v; j->fout[i] = 1; }
        else { j->vout[i] = miss; j->fout[i] = 0; }
    }
    return NULL;
}

/* lookup batch split evenly over `threads` threads (1 = the calling thread) */
void bpt_lookup_batch(const bptree* t, const u64* q, u64 B, u64* vout, uint8_t* fout, int threads) {
    if (threads <= 1 || B < (u64)threads) {
        lk_job j = { t, q, 0, B, vout, fout };
        lk_worker(&j);
        return;
    }
    pthread_t* th = malloc(sizeof(pthread_t) * threads);
    lk_job* jobs = malloc(sizeof(lk_job) * threads);
    for (int i = 0; i < threads; i++) {
        jobs[i] = (lk_job){ t, q, (u64)i * B / threads, (u64)(i + 1) * B / threads, vout, fout };
        pthread_create(&th[i], NULL, lk_worker, &jobs[i]);
    }
    for (int i = 0; i < threads; i++) pthread_join(th[i], NULL);
    free(th); free(jobs);
}

/*
 * Timed lookup batches for the CPU baseline (the paper times its CPU tree
 * with the batch split evenly over the threads, Section V-F, and a steady
 * clock, Section V-C).  nb batches of B queries, q[b*B .. b*B+B), each split
 * evenly over `threads` threads that are created once: the threads meet at a
 * barrier before and after every batch, and the calling thread (worker 0)
 * reads CLOCK_MONOTONIC at both, so times_ns[b] covers exactly batch b's
 * lookups plus one barrier.  Results as bpt_lookup_batch.  Returns 0, or -1
 * if the threads could not be started.
 */
typedef struct {
    pthread_mutex_t mu; pthread_cond_t cv; int go;   /* 1 run, -1 abort */
    pthread_barrier_t bar;
} pool_gate;

typedef struct {
    const bptree* t; const u64* q; u64 nb, B; u64* vout; uint8_t* fout;
    int T, id; pool_gate* g; u64* times;
} pool_job;

static u64 now_ns(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (u64)ts.tv_sec * 1000000000ull + (u64)ts.tv_nsec;
}

static void* pool_worker(void* p) {
    pool_job* j = p;
    pthread_mutex_lock(&j->g->mu);
    while (j->g->go == 0) pthread_cond_wait(&j->g->cv, &j->g->mu);
    int go = j->g->go;
    pthread_mutex_unlock(&j->g->mu);
    if (go < 0) return NULL;
    for (u64 b = 0; b < j->nb; b++) {
        u64 t0 = 0;
        pthread_barrier_wait(&j->g->bar);
        if (j->id == 0) t0 = now_ns();
        u64 base = b * j->B;
        lk_job w = { j->t, j->q + base, (u64)j->id * j->B / j->T, (u64)(j->id + 1) * j->B / j->T,
                     j->vout + base, j->fout + base };
        lk_worker(&w);
        pthread_barrier_wait(&j->g->bar);
        if (j->id == 0) j->times[b] = now_ns() - t0;
    }
    return NULL;
}

int bpt_lookup_batches_timed(const bptree* t, const u64* q, u64 nb, u64 B, u64* vout, uint8_t* fout,
                             int threads, u64* times_ns) {
    if (threads < 1) threads = 1;
    pool_gate g;
    pthread_mutex_init(&g.mu, NULL);
    pthread_cond_init(&g.cv, NULL);
    g.go = 0;
    pthread_barrier_init(&g.bar, NULL, (unsigned)threads);
    pthread_t* th = malloc(sizeof(pthread_t) * threads);
    pool_job* jobs = malloc(sizeof(pool_job) * threads);
    int started = 1;
    for (int i = 0; i < threads; i++)
        jobs[i] = (pool_job){ t, q, nb, B, vout, fout, threads, i, &g, times_ns };
    for (int i = 1; i < threads; i++) {
        if (pthread_create(&th[i], NULL, pool_worker, &jobs[i]) != 0) break;
        started++;
    }
    /* every thread must be running before any reaches the barrier */
    pthread_mutex_lock(&g.mu);
    g.go = started == threads ? 1 : -1;
    pthread_cond_broadcast(&g.cv);
    pthread_mutex_unlock(&g.mu);
    if (g.go > 0) pool_worker(&jobs[0]);
    for (int i = 1; i < started; i++) pthread_join(th[i], NULL);
    int rc = g.go > 0 ? 0 : -1;
    pthread_barrier_destroy(&g.bar);
    pthread_cond_destroy(&g.cv);
    pthread_mutex_destroy(&g.mu);
    free(th); free(jobs);
    return rc;
}

/* range via the leaf chain; same contract as ora_range */
void bpt_range_batch(const bptree* t, const u64* lo, const u64* hi, const u32* maxc, const u64* off,
                     u64 B, u64* out_keys, u64* out_vals, u32* count) {
    for (u64 i = 0; i < B; i++) {
        const bnode* x = t->root;
        while (!x->leaf) x = x->child[route(x, lo[i])];
        u32 c = 0;
        int p = 0;
        while (p < x->n && x->key[p] < lo[i]) p++;
        while (x && c < maxc[i] && lo[i] <= hi[i]) {
            if (p >= x->n) { x = x->next; p = 0; continue; }
            if (x->key[p] > hi[i]) break;
            out_keys[off[i] + c] = x->key[p]; out_vals[off[i] + c] = x->val[p];
            c++; p++;
        }
        count[i] = c;
    }
}

/*
 * Level-wise batch search (Sections IV-A and IV-F), the paper's traversal
 * written out on the pointer tree.  The batch sq[0..B) must be ascending.
 * A FIFO holds one tree level as entries (node, number of keys); the keys
 * are taken in order by one running key index.  For each entry the node is
 * taken once and its keys are compared with it one after another: at an
 * inner node each key yields a child, and a key whose child equals that of
 * the entry written last to the next FIFO increments that entry's count,
 * otherwise it opens a new entry with count 1.  At the leaves each key's
 * result (its value, or -1 with found = 0, Section IV-D) is written in
 * processing order.
 *
 * Each entry is reported as a run: (level, first key index, count, node
 * identity), levels in order.  Returns the number of runs, or -1 if the
 * batch is not ascending or more than run_cap runs would be written.
 */
long long bpt_levelwise(const bptree* t, const u64* sq, u64 B, u64* vout, uint8_t* fout, u32* run_level,
                        u64* run_first, u64* run_count, u64* run_node, u64 run_cap) {
    for (u64 i = 1; i < B; i++)
        if (sq[i] < sq[i - 1]) return -1;
    typedef struct { const bnode* x; u64 n; } entry;
    entry* cur = malloc(sizeof(entry) * (B ? B : 1));
    entry* nxt = malloc(sizeof(entry) * (B ? B : 1));
    u64 ncur = 0, w = 0;
    long long ret = 0;
    const u64 miss = ones(t->width);
    if (B) cur[ncur++] = (entry){ t->root, B };
    for (int level = 0; level < t->height && ret == 0; level++) {
        u64 idx = 0, nn = 0;
        for (u64 e = 0; e < ncur; e++) {
            const bnode* x = cur[e].x;
            if (w >= run_cap) { ret = -1; break; }
            run_level[w] = (u32)level;
            run_first[w] = idx;
            run_count[w] = cur[e].n;
            run_node[w] = (u64)(uintptr_t)x;
            w++;
            for (u64 j = 0; j < cur[e].n; j++, idx++) {
                const u64 k = sq[idx];
                if (x->leaf) {
                    int p = 0;
                    while (p < x->n && x->key[p] != k) p++;
                    if (p < x->n) { vout[idx] = x->val[p]; fout[idx] = 1; }
                    else { vout[idx] = miss; fout[idx] = 0; }
                } else {
                    const bnode* c = x->child[route(x, k)];
                    if (nn > 0 && nxt[nn - 1].x == c) nxt[nn - 1].n++;
                    else nxt[nn++] = (entry){ c, 1 };
                }
            }
        }
        entry* tmp = cur; cur = nxt; nxt = tmp;
        ncur = nn;
    }
    free(cur);
    free(nxt);
    return ret == 0 ? (long long)w : -1;
}

void bpt_stats(const bptree* t, u64* out /* height, n_keys, n_inner, n_leaves */) {
    out[0] = (u64)t->height; out[1] = t->n_keys; out[2] = t->n_inner; out[3] = t->n_leaves;
}

/* ------------------------------------------------------ export format -- */
/*
 * Header (48 bytes, little endian):
 *   u32 magic 0x58455447, key_bytes, fanout, leaf_cap, height, root,
 *   first_leaf, n_inner, n_leaves, reserved; u64 n_keys
 * then n_inner inner records:  key[fanout] (key_bytes each), child[fanout] (u32)
 * then n_leaves leaf records:  key[leaf_cap], val[leaf_cap] (key_bytes each),
 *                              u32 count, u32 next
 * A node reference has bit 31 set for a leaf (index in the low 31 bits), is
 * an inner index otherwise; 0xFFFFFFFF is "none".  Inner padding: entry slots
 * >= children-1 hold the largest key, child slots >= children hold none.
 * Leaf padding: key slots >= count repeat the last key (largest key when
 * count = 0).
 */
#define EX_MAGIC 0x58455447u
#define REF_NONE 0xFFFFFFFFu
#define REF_LEAF 0x80000000u

typedef struct { u64 n_inner, n_leaves; } ex_sizes;

static void put_key(uint8_t* p, u64 k, int kb) { if (kb == 4) { u32 x = (u32)k; memcpy(p, &x, 4); } else memcpy(p, &k, 8); }
static u64 get_key(const uint8_t* p, int kb) { if (kb == 4) { u32 x; memcpy(&x, p, 4); return x; } u64 x; memcpy(&x, p, 8); return x; }

u64 bpt_export_bytes(const bptree* t) {
    int kb = t->width / 8;
    return 48 + t->n_inner * (u64)(t->fanout * (kb + 4)) + t->n_leaves * (u64)(t->cap * 2 * kb + 8);
}

/*
 * Serialise: inner nodes numbered in breadth-first order, leaves in chain
 * order.  Returns bytes written or 0 if the buffer is too small.
 */
u64 bpt_export(const bptree* t, uint8_t* buf, u64 bytes) {
    u64 need = bpt_export_bytes(t);
    if (bytes < need) return 0;
    int kb = t->width / 8, F = t->fanout, C = t->cap;
    u64 ni = t->n_inner, nl = t->n_leaves;
    u64 rin = (u64)F * (kb + 4), rlf = (u64)C * 2 * kb + 8;
    uint8_t* inner = buf + 48;
    uint8_t* leaves = inner + ni * rin;
    u64 maxk = ones(t->width);
    /* BFS over inner nodes; leaves numbered by chain order */
    bnode** q = malloc(sizeof(bnode*) * (ni + 1));
    u64 qh = 0, qt = 0;
    const bnode* first = t->root;
    while (!first->leaf) first = first->child[0];
    /* leaf ids: walk the chain once and stash the index in a temporary map */
    u64 li = 0;
    bnode** lmap = malloc(sizeof(bnode*) * (nl + 1));
    for (bnode* x = (bnode*)first; x; x = x->next) { x->tag = li; lmap[li++] = x; }
    if (!t->root->leaf) q[qt++] = t->root;
    u64 next_inner_id = qt;
    while (qh < qt) {
        bnode* x = q[qh];
        uint8_t* rec = inner + qh * rin;
        for (int i = 0; i < F; i++) put_key(rec + (u64)i * kb, i < x->n - 1 ? x->key[i] : maxk, kb);
        u32* ch = (u32*)(rec + (u64)F * kb);
        for (int i = 0; i < F; i++) {
            u32 r = REF_NONE;
            if (i < x->n) {
                bnode* c = x->child[i];
                if (c->leaf) {
                    r = REF_LEAF | (u32)c->tag;
                } else {
                    r = (u32)next_inner_id++;
                    q[qt++] = c;
                }
            }
            memcpy(&ch[i], &r, 4);
        }
        qh++;
    }
    for (u64 id = 0; id < li; id++) {
        bnode* x = lmap[id];
        uint8_t* rec = leaves + id * rlf;
        for (int i = 0; i < C; i++) {
            u64 k = i < x->n ? x->key[i] : (x->n ? x->key[x->n - 1] : maxk);
            put_key(rec + (u64)i * kb, k, kb);
            put_key(rec + (u64)(C + i) * kb, i < x->n ? x->val[i] : maxk, kb);
        }
        u32 cnt = (u32)x->n, nx = (id + 1 < li) ? (u32)(id + 1) : REF_NONE;
        memcpy(rec + (u64)2 * C * kb, &cnt, 4);
        memcpy(rec + (u64)2 * C * kb + 4, &nx, 4);
    }
    u32 hdr[10] = { EX_MAGIC, (u32)kb, (u32)F, (u32)C, (u32)t->height,
                    t->root->leaf ? (REF_LEAF | 0u) : 0u, 0u, (u32)qt, (u32)li, 0u };
    memcpy(buf, hdr, 40);
    memcpy(buf + 40, &t->n_keys, 8);
    free(q); free(lmap);
    return need;
}

/* ------------------------------------------------------------------ O4 -- */

/* violation bits */
#define V_FORMAT    (1u << 0)  /* bad header or sizes */
#define V_SORTED    (1u << 1)  /* I1 leaf keys / chain not strictly ascending */
#define V_DEPTH     (1u << 2)  /* I2 leaves at unequal depth, or != height */
#define V_FILL      (1u << 3)  /* I3 node fill out of bounds */
#define V_COUNT     (1u << 4)  /* I4 key count differs from header */
#define V_SEPARATOR (1u << 5)  /* I5 key outside its separator interval */
#define V_CHAIN     (1u << 6)  /* I6 chain order or termination wrong */
#define V_REACH     (1u << 7)  /* I7 node reached twice or out of range */
#define V_PADDING   (1u << 8)  /* padding rule broken */

typedef struct {
    const uint8_t* inner; const uint8_t* leaves;
    int kb, vb, F, C; u64 ni, nl, rin, rlf;
    uint8_t maxk[32];                  /* the largest key: kb bytes of 0xFF */
    uint8_t* seen_i; uint8_t* seen_l;
    u32* leaf_order; u64 n_order;      /* leaves in in-order traversal */
    /* in-order output: keys as u64 (kb <= 8) or as kb packed bytes */
    u64* out_keys; uint8_t* out_kbytes; u64* out_vals; u64 out_cap; u64 n_out;
    const uint8_t* prev_key;           /* last key emitted (I1 across leaves) */
    u32 viol; int height;
} chk;

/* keys of 4 or 8 bytes are little-endian unsigned integers; longer keys
 * compare as byte strings (the byte-key order above) */
static int kcmp(const chk* c, const uint8_t* a, const uint8_t* b) {
    if (c->kb <= 8) { u64 x = get_key(a, c->kb), y = get_key(b, c->kb); return x < y ? -1 : x > y; }
    return memcmp(a, b, (size_t)c->kb);
}
static const uint8_t* ik(const chk* c, u64 node, int i) { return c->inner + node * c->rin + (u64)i * c->kb; }
static u32 ic(const chk* c, u64 node, int i) { u32 r; memcpy(&r, c->inner + node * c->rin + (u64)c->F * c->kb + (u64)i * 4, 4); return r; }
static const uint8_t* lk(const chk* c, u64 leaf, int i) { return c->leaves + leaf * c->rlf + (u64)i * c->kb; }
static u64 lv(const chk* c, u64 leaf, int i) { return get_key(c->leaves + leaf * c->rlf + (u64)c->C * c->kb + (u64)i * c->vb, c->vb); }
static u32 lcnt(const chk* c, u64 leaf) { u32 r; memcpy(&r, c->leaves + leaf * c->rlf + (u64)c->C * (c->kb + c->vb), 4); return r; }
static u32 lnext(const chk* c, u64 leaf) { u32 r; memcpy(&r, c->leaves + leaf * c->rlf + (u64)c->C * (c->kb + c->vb) + 4, 4); return r; }

static void emit(chk* c, const uint8_t* k, u64 v) {
    if (c->prev_key && kcmp(c, c->prev_key, k) >= 0) c->viol |= V_SORTED;   /* I1 across leaves */
    c->prev_key = k;
    if (c->n_out < c->out_cap) {
        if (c->out_keys) c->out_keys[c->n_out] = get_key(k, c->kb);
        else memcpy(c->out_kbytes + c->n_out * c->kb, k, (size_t)c->kb);
        c->out_vals[c->n_out] = v;
    }
    c->n_out++;
}

/*
 * Visit node `ref` at depth d (root = 1).  Every key below must satisfy
 * lo < key <= hi; a null bound is absent.
 */
static void visit(chk* c, u32 ref, int d, int is_root, int many_leaves, const uint8_t* lo, const uint8_t* hi) {
    if (ref == REF_NONE) { c->viol |= V_REACH; return; }
    if (ref & REF_LEAF) {
        u64 id = ref & ~REF_LEAF;
        if (id >= c->nl) { c->viol |= V_REACH; return; }
        if (c->seen_l[id]) { c->viol |= V_REACH; return; }
        c->seen_l[id] = 1;
        c->leaf_order[c->n_order++] = (u32)id;
        if (d != c->height) c->viol |= V_DEPTH;
        u32 n = lcnt(c, id);
        if (n > (u32)c->C) { c->viol |= V_FILL; n = (u32)c->C; }
        if (many_leaves && n < (u32)((c->C + 1) / 2)) c->viol |= V_FILL;
        for (u32 i = 0; i < n; i++) {
            const uint8_t* k = lk(c, id, (int)i);
            if (i && kcmp(c, lk(c, id, (int)i - 1), k) >= 0) c->viol |= V_SORTED;
            if ((lo && kcmp(c, k, lo) <= 0) || (hi && kcmp(c, k, hi) > 0)) c->viol |= V_SEPARATOR;
            emit(c, k, lv(c, id, (int)i));
        }
        const uint8_t* pad = n ? lk(c, id, (int)n - 1) : c->maxk;
        for (u32 i = n; i < (u32)c->C; i++) if (kcmp(c, lk(c, id, (int)i), pad) != 0) c->viol |= V_PADDING;
        return;
    }
    if (ref >= c->ni) { c->viol |= V_REACH; return; }
    if (c->seen_i[ref]) { c->viol |= V_REACH; return; }
    c->seen_i[ref] = 1;
    if (d >= c->height) { c->viol |= V_DEPTH; return; }
    int n = 0;
    while (n < c->F && ic(c, ref, n) != REF_NONE) n++;
    for (int i = n; i < c->F; i++) if (ic(c, ref, i) != REF_NONE) c->viol |= V_PADDING;
    /* Section III: a non-root inner node has at least m/2 children, an
       inner root at least two */
    if (is_root ? n < 2 : n < (c->F + 1) / 2) c->viol |= V_FILL;
    for (int i = n - 1 < 0 ? 0 : n - 1; i < c->F; i++) if (kcmp(c, ik(c, ref, i), c->maxk) != 0) c->viol |= V_PADDING;
    for (int i = 0; i + 1 < n; i++) {
        const uint8_t* sp = ik(c, ref, i);
        if ((lo && kcmp(c, sp, lo) <= 0) || (hi && kcmp(c, sp, hi) > 0)) c->viol |= V_SEPARATOR;
        if (i && kcmp(c, ik(c, ref, i - 1), sp) >= 0) c->viol |= V_SEPARATOR;
    }
    for (int i = 0; i < n; i++) {
        const uint8_t* clo = i ? ik(c, ref, i - 1) : lo;
        const uint8_t* chi = (i + 1 < n) ? ik(c, ref, i) : hi;
        visit(c, ic(c, ref, i), d + 1, 0, many_leaves, clo, chi);
    }
}

/*
 * Check an exported tree whose keys are kb = 4, 8 or 32 bytes.  The header's
 * last u32 (reserved in the library's 4/8-byte format) gives the value
 * width: 0 means the key width; 32-byte keys carry 8-byte values.  Leaf
 * records are key[leaf_cap] (kb each), value[leaf_cap] (vb each), u32 count,
 * u32 next.  The in-order pairs go to out_keys (u64, when kb <= 8) or
 * out_kbytes (kb packed bytes each) and out_vals, up to out_cap of them;
 * *n_out receives how many the tree holds.  Returns the violation bits
 * (0 = all invariants hold).
 */
static u32 check_export(const uint8_t* buf, u64 bytes, u64* out_keys, uint8_t* out_kbytes, u64* out_vals,
                        u64 out_cap, u64* n_out, int* kb_out) {
    *n_out = 0;
    if (bytes < 48) return V_FORMAT;
    u32 hdr[10]; u64 nk;
    memcpy(hdr, buf, 40); memcpy(&nk, buf + 40, 8);
    u32 kb = hdr[1], vb = hdr[9] ? hdr[9] : hdr[1];
    int ok_width = ((kb == 4 || kb == 8) && vb == kb) || (kb == 32 && vb == 8);
    if (hdr[0] != EX_MAGIC || !ok_width || hdr[2] < 4 || hdr[2] > 1024 || hdr[3] < 2 || hdr[3] > 1024 ||
        hdr[4] < 1) return V_FORMAT;
    if (kb_out) *kb_out = (int)kb;
    if ((kb > 8) != (out_kbytes != NULL)) return V_FORMAT;
    chk c;
    memset(&c, 0, sizeof c);
    c.kb = (int)kb; c.vb = (int)vb; c.F = (int)hdr[2]; c.C = (int)hdr[3]; c.height = (int)hdr[4];
    c.ni = hdr[7]; c.nl = hdr[8];
    c.rin = (u64)c.F * (c.kb + 4); c.rlf = (u64)c.C * (c.kb + c.vb) + 8;
    if (48 + c.ni * c.rin + c.nl * c.rlf > bytes) return V_FORMAT;
    c.inner = buf + 48; c.leaves = c.inner + c.ni * c.rin;
    memset(c.maxk, 0xFF, sizeof c.maxk);
    c.seen_i = calloc(c.ni + 1, 1); c.seen_l = calloc(c.nl + 1, 1);
    c.leaf_order = malloc(sizeof(u32) * (c.nl + 1));
    c.out_keys = out_keys; c.out_kbytes = out_kbytes; c.out_vals = out_vals; c.out_cap = out_cap;
    u32 root = hdr[5];
    int many = (root & REF_LEAF) == 0 || root == REF_NONE;
    visit(&c, root, 1, 1, many, NULL, NULL);
    /* I4 */
    if (c.n_out != nk) c.viol |= V_COUNT;
    /* I6: the chain from first_leaf must equal the in-order leaf sequence */
    u32 x = hdr[6];
    u64 steps = 0;
    for (; x != REF_NONE && steps <= c.nl; steps++) {
        if (x >= c.nl || steps >= c.n_order || c.leaf_order[steps] != x) { c.viol |= V_CHAIN; break; }
        x = lnext(&c, x);
    }
    if (!(c.viol & V_CHAIN) && (x != REF_NONE || steps != c.n_order)) c.viol |= V_CHAIN;
    *n_out = c.n_out;
    free(c.seen_i); free(c.seen_l); free(c.leaf_order);
    return c.viol;
}

/* 4- and 8-byte keys: the in-order keys and values as u64 */
u32 ora_check_export(const uint8_t* buf, u64 bytes, u64* out_keys, u64* out_vals, u64 out_cap, u64* n_out) {
    if (bytes >= 8) { u32 kb; memcpy(&kb, buf + 4, 4); if (kb > 8) { *n_out = 0; return V_FORMAT; } }
    return check_export(buf, bytes, out_keys, NULL, out_vals, out_cap, n_out, NULL);
}

/* 32-byte keys: the in-order keys as packed bytes, values as u64 */
u32 orb_check_export(const uint8_t* buf, u64 bytes, uint8_t* out_keys, u64* out_vals, u64 out_cap, u64* n_out) {
    if (bytes >= 8) { u32 kb; memcpy(&kb, buf + 4, 4); if (kb <= 8) { *n_out = 0; return V_FORMAT; } }
    return check_export(buf, bytes, NULL, out_keys, out_vals, out_cap, n_out, NULL);
}
