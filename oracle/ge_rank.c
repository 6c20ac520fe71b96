/*
 * Oracle (test infrastructure only): rank of a sparse integer matrix over
 * GF(p) by sparse Gaussian elimination, in plain C.
 *
 * This is the plain definition of the value the block Wiedemann rank algorithm
 * returns (Section 2.5, "Block Wiedemann Rank Algorithm"), written as ordinary
 * elimination so that it can run at mid-size (a few million non-zeros), where
 * the Python twin in ge.py is too slow.  Every arithmetic step reduces with a
 * fresh "% p"; there is no delayed reduction and nothing is shared with the
 * GPU library.
 *
 * Pivoting (Markowitz-style, to limit fill): two candidates are formed, (A) a
 * shortest remaining row with its column held by the fewest remaining rows,
 * and (B) a column held by the fewest remaining rows with its shortest row;
 * the one with the smaller (row length - 1) * (column count - 1) is taken.
 * The chosen column is eliminated from every other remaining row and the
 * pivot row is dropped.  The rank is the number of pivots.  The pivot order
 * affects only speed, never the rank.
 *
 * Pinned (tests) against the Python sparse and dense eliminations and Bareiss
 * over Q on random small matrices, and against planted ranks.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t *col;
    uint32_t *val;
    int32_t len, cap;
    int32_t active;
} row_t;

typedef struct {
    int32_t *rows;
    int32_t len, cap;
    int32_t count; /* remaining rows holding this column */
} col_t;

typedef struct {
    int64_t key; /* (len << 32) | row */
} heap_ent;

static uint64_t powmod(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = (r * a) % p;
        a = (a * a) % p;
        e >>= 1;
    }
    return r;
}

static int col_push(col_t *c, int32_t r) {
    if (c->len == c->cap) {
        int32_t nc = c->cap ? 2 * c->cap : 4;
        int32_t *nr = (int32_t *)realloc(c->rows, sizeof(int32_t) * (size_t)nc);
        if (!nr) return -1;
        c->rows = nr;
        c->cap = nc;
    }
    c->rows[c->len++] = r;
    return 0;
}

/* binary min-heap on int64 keys */
typedef struct {
    int64_t *a;
    int64_t len, cap;
} heap_t;

static int heap_push(heap_t *h, int64_t k) {
    if (h->len == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        int64_t *na = (int64_t *)realloc(h->a, sizeof(int64_t) * (size_t)nc);
        if (!na) return -1;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->len++;
    h->a[i] = k;
    while (i > 0) {
        int64_t par = (i - 1) / 2;
        if (h->a[par] <= h->a[i]) break;
        int64_t t = h->a[par];
        h->a[par] = h->a[i];
        h->a[i] = t;
        i = par;
    }
    return 0;
}

static int64_t heap_pop(heap_t *h) {
    int64_t top = h->a[0];
    h->a[0] = h->a[--h->len];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < h->len && h->a[l] < h->a[s]) s = l;
        if (r < h->len && h->a[r] < h->a[s]) s = r;
        if (s == i) break;
        int64_t t = h->a[s];
        h->a[s] = h->a[i];
        h->a[i] = t;
        i = s;
    }
    return top;
}

static int32_t row_find(const row_t *r, int32_t c) {
    int32_t lo = 0, hi = r->len - 1;
    while (lo <= hi) {
        int32_t mid = (lo + hi) / 2;
        if (r->col[mid] == c) return mid;
        if (r->col[mid] < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/*
 * Returns the rank (>= 0), or -1 on allocation failure / bad input.
 * row_ptr: m+1 offsets; col_idx, val: nnz entries (duplicates are summed).
 */
int64_t oracle_rank_modp(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                         const int32_t *val, uint32_t p) {
    if (m < 0 || n < 0 || p < 2) return -1;
    if (m >= (1LL << 31) || n >= (1LL << 31)) return -1;
    row_t *rows = (row_t *)calloc((size_t)(m ? m : 1), sizeof(row_t));
    col_t *cols = (col_t *)calloc((size_t)(n ? n : 1), sizeof(col_t));
    heap_t heap = {0, 0, 0};
    heap_t cheap = {0, 0, 0};
    int32_t *tmpc = NULL;
    uint32_t *tmpv = NULL;
    int64_t tmpcap = 0;
    int64_t rank = -1;
    if (!rows || !cols) goto done;

    /* load rows: sort each row's entries by column, sum duplicates mod p */
    for (int64_t i = 0; i < m; i++) {
        int64_t b = row_ptr[i], e = row_ptr[i + 1];
        int32_t cnt = (int32_t)(e - b);
        row_t *r = &rows[i];
        r->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt ? cnt : 1));
        r->val = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cnt ? cnt : 1));
        if (!r->col || !r->val) goto done;
        r->cap = cnt ? cnt : 1;
        /* insertion sort (rows are short) */
        int32_t len = 0;
        for (int64_t t = b; t < e; t++) {
            int32_t c = col_idx[t];
            if (c < 0 || c >= n) goto done;
            int64_t v = (int64_t)val[t] % (int64_t)p;
            if (v < 0) v += p;
            int32_t pos = len;
            while (pos > 0 && r->col[pos - 1] > c) pos--;
            if (pos > 0 && r->col[pos - 1] == c) {
                r->val[pos - 1] = (uint32_t)(((uint64_t)r->val[pos - 1] + (uint64_t)v) % p);
                continue;
            }
            memmove(r->col + pos + 1, r->col + pos, sizeof(int32_t) * (size_t)(len - pos));
            memmove(r->val + pos + 1, r->val + pos, sizeof(uint32_t) * (size_t)(len - pos));
            r->col[pos] = c;
            r->val[pos] = (uint32_t)v;
            len++;
        }
        /* drop zeros */
        int32_t w = 0;
        for (int32_t t = 0; t < len; t++)
            if (r->val[t]) {
                r->col[w] = r->col[t];
                r->val[w] = r->val[t];
                w++;
            }
        r->len = w;
        r->active = w > 0;
        for (int32_t t = 0; t < w; t++) {
            if (col_push(&cols[r->col[t]], (int32_t)i)) goto done;
            cols[r->col[t]].count++;
        }
        if (w && heap_push(&heap, ((int64_t)w << 32) | i)) goto done;
    }

    for (int64_t c = 0; c < n; c++)
        if (cols[c].count && heap_push(&cheap, ((int64_t)cols[c].count << 32) | c)) goto done;

    rank = 0;
    for (;;) {
        /* candidate A: a shortest remaining row and its sparsest column */
        int32_t ia = -1, ca = -1;
        while (heap.len) {
            int64_t key = heap.a[0];
            int32_t i = (int32_t)(key & 0xffffffff);
            if (!rows[i].active || rows[i].len != (int32_t)(key >> 32)) { heap_pop(&heap); continue; }
            ia = i;
            break;
        }
        if (ia < 0) break;
        {
            row_t *r = &rows[ia];
            int32_t best = 0;
            for (int32_t t = 1; t < r->len; t++) {
                int32_t a = r->col[t], bb = r->col[best];
                if (cols[a].count < cols[bb].count || (cols[a].count == cols[bb].count && a < bb)) best = t;
            }
            ca = r->col[best];
        }
        int64_t cost_a = (int64_t)(rows[ia].len - 1) * (cols[ca].count - 1);
        /* candidate B: a sparsest remaining column and its shortest row */
        int32_t ib = -1, cb = -1;
        while (cost_a > 0 && cheap.len) {
            int64_t key = cheap.a[0];
            int32_t c = (int32_t)(key & 0xffffffff);
            if (cols[c].count == 0 || cols[c].count != (int32_t)(key >> 32)) {
                heap_pop(&cheap);
                if (cols[c].count) heap_push(&cheap, ((int64_t)cols[c].count << 32) | c);
                continue;
            }
            cb = c;
            break;
        }
        if (cb >= 0) {
            col_t *cc0 = &cols[cb];
            for (int32_t q = 0; q < cc0->len; q++) {
                int32_t j = cc0->rows[q];
                if (!rows[j].active || row_find(&rows[j], cb) < 0) continue;
                if (ib < 0 || rows[j].len < rows[ib].len || (rows[j].len == rows[ib].len && j < ib)) ib = j;
            }
        }
        int32_t i, pcol;
        if (ib >= 0 && (int64_t)(rows[ib].len - 1) * (cols[cb].count - 1) < cost_a) {
            i = ib;
            pcol = cb;
        } else {
            i = ia;
            pcol = ca;
        }
        row_t *pr = &rows[i];
        int32_t best = row_find(pr, pcol);
        int32_t pc = pcol;
        uint64_t inv = powmod(pr->val[best], p - 2, p);
        pr->active = 0;
        for (int32_t t = 0; t < pr->len; t++) {
            int32_t c0 = pr->col[t];
            if (--cols[c0].count > 0 && heap_push(&cheap, ((int64_t)cols[c0].count << 32) | c0)) {
                rank = -1;
                goto done;
            }
        }
        rank++;
        col_t *cc = &cols[pc];
        for (int32_t q = 0; q < cc->len; q++) {
            int32_t j = cc->rows[q];
            row_t *rj = &rows[j];
            if (!rj->active) continue;
            int32_t pos = row_find(rj, pc);
            if (pos < 0) continue;
            uint64_t f = ((uint64_t)rj->val[pos] * inv) % p;
            /* merged = rj - f * pr */
            int64_t need = (int64_t)rj->len + pr->len;
            if (need > tmpcap) {
                int64_t nc = need * 2;
                int32_t *nc1 = (int32_t *)realloc(tmpc, sizeof(int32_t) * (size_t)nc);
                if (!nc1) { rank = -1; goto done; }
                tmpc = nc1;
                uint32_t *nv1 = (uint32_t *)realloc(tmpv, sizeof(uint32_t) * (size_t)nc);
                if (!nv1) { rank = -1; goto done; }
                tmpv = nv1;
                tmpcap = nc;
            }
            int32_t a = 0, b = 0, w = 0;
            while (a < rj->len || b < pr->len) {
                int32_t ca = a < rj->len ? rj->col[a] : INT32_MAX;
                int32_t cb = b < pr->len ? pr->col[b] : INT32_MAX;
                if (ca < cb) {
                    tmpc[w] = ca;
                    tmpv[w++] = rj->val[a++];
                } else if (cb < ca) {
                    uint64_t v = (p - ((f * pr->val[b]) % p)) % p;
                    if (v) {
                        tmpc[w] = cb;
                        tmpv[w++] = (uint32_t)v;
                        if (col_push(&cols[cb], j)) { rank = -1; goto done; }
                        cols[cb].count++;
                    }
                    b++;
                } else {
                    uint64_t v = ((uint64_t)rj->val[a] + p - ((f * pr->val[b]) % p)) % p;
                    if (v) {
                        tmpc[w] = ca;
                        tmpv[w++] = (uint32_t)v;
                    } else if (--cols[ca].count > 0 &&
                               heap_push(&cheap, ((int64_t)cols[ca].count << 32) | ca)) {
                        rank = -1;
                        goto done;
                    }
                    a++;
                    b++;
                }
            }
            if (w > rj->cap) {
                int32_t *nc1 = (int32_t *)realloc(rj->col, sizeof(int32_t) * (size_t)w);
                if (!nc1) { rank = -1; goto done; }
                rj->col = nc1;
                uint32_t *nv1 = (uint32_t *)realloc(rj->val, sizeof(uint32_t) * (size_t)w);
                if (!nv1) { rank = -1; goto done; }
                rj->val = nv1;
                rj->cap = w;
            }
            memcpy(rj->col, tmpc, sizeof(int32_t) * (size_t)w);
            memcpy(rj->val, tmpv, sizeof(uint32_t) * (size_t)w);
            rj->len = w;
            if (w == 0) rj->active = 0;
            else if (heap_push(&heap, ((int64_t)w << 32) | j)) { rank = -1; goto done; }
        }
        cc->len = 0;
    }

done:
    if (rows)
        for (int64_t i = 0; i < m; i++) {
            free(rows[i].col);
            free(rows[i].val);
        }
    if (cols)
        for (int64_t c = 0; c < n; c++) free(cols[c].rows);
    free(rows);
    free(cols);
    free(heap.a);
    free(cheap.a);
    free(tmpc);
    free(tmpv);
    return rank;
}
