/*
 * rsa_oracle.c -- serial CPU oracle for RSA of linear k-mers on an L x L
 * torus (arXiv:1810.06800).  Plain C, one sample at a time, no threads.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load or call this library.  It shares no code
 * with the GPU library.  See rsa_oracle.h for the definition being computed.
 *
 * Written for obviousness, not speed: the next placement is found by counting
 * available placements row by row in canonical order; blocked placements are
 * cleared exactly as the definition says (every placement that covers one of
 * the new sites); clusters are kept the way Sec. II.C-II.E describe them
 * (per-k-mer cluster id and displacement from the cluster root, the smaller
 * cluster relabelled on a merge).
 */
#include "rsa_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------
 * Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two
 * 32x32->64 multiplies; the key is bumped by the Weyl constants between
 * rounds.
 * ------------------------------------------------------------------------- */
void rsao_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mult0 = 0xD2511F53u, mult1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint64_t p0 = (uint64_t)mult0 * x0;
        uint64_t p1 = (uint64_t)mult1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* SplitMix64 output finalizer (Steele, Lea, Flood, OOPSLA'14). */
uint64_t rsao_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* rank = floor(u * a / 2^64): a uniform integer in [0, a). */
uint32_t rsao_rank(uint64_t u, uint32_t a)
{
    unsigned __int128 prod = (unsigned __int128)u * (unsigned __int128)a;
    return (uint32_t)(prod >> 64);
}

/* ------------------------------------------------------------------------- */

typedef struct {
    uint32_t L, k, Wd;          /* Wd = 64-bit words per bitmap row          */
    int32_t *map;               /* site -> k-mer id, -1 when empty           */
    uint64_t *avail[2];         /* avail[o][y*Wd + x/64] bit x%64            */
    int64_t *cnt;               /* available placements per row: [o*L + y]   */
    uint64_t A;                 /* available placements in total             */
    /* per k-mer (index = deposit number t) */
    uint32_t *anchor;           /* site index y*L + x of the first site      */
    uint8_t *orient;            /* 0 = H, 1 = V                              */
    int64_t *cid;               /* cluster id (the id of some member k-mer)  */
    int64_t *dx, *dy;           /* anchor minus the cluster root's anchor,   */
                                /* unwrapped (Sec. II.D)                      */
    int64_t *next;              /* next member of the same cluster, or -1    */
    /* per cluster (indexed by cluster id) */
    int64_t *head, *tail, *size;
    uint8_t *wx, *wy;           /* the cluster wraps in x / in y             */
    uint64_t cap;               /* capacity of the per-k-mer arrays          */
    uint64_t wchg;              /* availability words changed so far         */
} sample_t;

static void free_sample(sample_t *s)
{
    free(s->map); free(s->avail[0]); free(s->avail[1]); free(s->cnt);
    free(s->anchor); free(s->orient); free(s->cid); free(s->dx); free(s->dy);
    free(s->next); free(s->head); free(s->tail); free(s->size); free(s->wx); free(s->wy);
}

static int64_t mod_l(int64_t a, int64_t L)
{
    int64_t r = a % L;
    return r < 0 ? r + L : r;
}

static int popcount64(uint64_t w)
{
    return __builtin_popcountll(w);
}

/* Initial state: every placement available (vertical ones too unless
 * H_ONLY), every site empty (Sec. II.A). */
static int init_sample(sample_t *s, const rsao_desc_t *d)
{
    memset(s, 0, sizeof(*s));
    uint64_t L = d->L;
    s->L = d->L;
    s->k = d->k;
    s->Wd = (uint32_t)((L + 63) / 64);
    s->cap = L * L / d->k + 1;
    s->map = (int32_t *)malloc(L * L * sizeof(int32_t));
    s->avail[0] = (uint64_t *)calloc(L * s->Wd, sizeof(uint64_t));
    s->avail[1] = (uint64_t *)calloc(L * s->Wd, sizeof(uint64_t));
    s->cnt = (int64_t *)calloc(2 * L, sizeof(int64_t));
    s->anchor = (uint32_t *)malloc(s->cap * sizeof(uint32_t));
    s->orient = (uint8_t *)malloc(s->cap);
    s->cid = (int64_t *)malloc(s->cap * sizeof(int64_t));
    s->dx = (int64_t *)malloc(s->cap * sizeof(int64_t));
    s->dy = (int64_t *)malloc(s->cap * sizeof(int64_t));
    s->next = (int64_t *)malloc(s->cap * sizeof(int64_t));
    s->head = (int64_t *)malloc(s->cap * sizeof(int64_t));
    s->tail = (int64_t *)malloc(s->cap * sizeof(int64_t));
    s->size = (int64_t *)malloc(s->cap * sizeof(int64_t));
    s->wx = (uint8_t *)malloc(s->cap);
    s->wy = (uint8_t *)malloc(s->cap);
    if (!s->map || !s->avail[0] || !s->avail[1] || !s->cnt || !s->anchor || !s->orient ||
        !s->cid || !s->dx || !s->dy || !s->next || !s->head || !s->tail || !s->size ||
        !s->wx || !s->wy) {
        free_sample(s);
        return RSAO_ENOMEM;
    }
    for (uint64_t i = 0; i < L * L; ++i) s->map[i] = -1;
    int norient = (d->flags & RSAO_FLAG_H_ONLY) ? 1 : 2;
    s->A = 0;
    for (int o = 0; o < norient; ++o) {
        for (uint64_t y = 0; y < L; ++y) {
            for (uint64_t x = 0; x < L; ++x)
                s->avail[o][y * s->Wd + x / 64] |= 1ull << (x % 64);
            s->cnt[o * L + y] = (int64_t)L;
            s->A += L;
        }
    }
    return RSAO_OK;
}

/* Placement with exactly `rank` available placements of smaller canonical
 * index: count row by row in canonical order (o, y), then word by word and
 * bit by bit inside the row.  Returns the canonical index. */
static uint32_t select_placement(const sample_t *s, uint64_t rank)
{
    uint64_t L = s->L;
    uint64_t row = 0;
    while (rank >= (uint64_t)s->cnt[row]) {
        rank -= (uint64_t)s->cnt[row];
        ++row;
    }
    uint32_t o = (uint32_t)(row / L), y = (uint32_t)(row % L);
    const uint64_t *words = s->avail[o] + (uint64_t)y * s->Wd;
    uint32_t w = 0;
    while (rank >= (uint64_t)popcount64(words[w])) {
        rank -= (uint64_t)popcount64(words[w]);
        ++w;
    }
    uint64_t word = words[w];
    for (uint32_t b = 0; b < 64; ++b) {
        if (word & (1ull << b)) {
            if (rank == 0) {
                uint64_t x = (uint64_t)w * 64 + b;
                return (uint32_t)((uint64_t)o * L * L + (uint64_t)y * L + x);
            }
            --rank;
        }
    }
    return 0xFFFFFFFFu; /* unreachable when the counts are right */
}

/* Bits of the cyclic column interval [c0, c0 + len) (mod L), len <= L, as a
 * list of (word, mask) pairs with each word listed once.  Columns are visited
 * in cyclic order, so a word seen before is either the previous column's
 * word or, after the seam, the word of c0 (the interval is shorter than L,
 * so the columns after the seam all lie below c0). */
static uint32_t interval_masks(uint32_t L, uint32_t c0, uint32_t len, uint32_t *words,
                               uint64_t *masks)
{
    uint32_t n = 0;
    for (uint32_t i = 0; i < len; ++i) {
        uint32_t c = (uint32_t)(((uint64_t)c0 + i) % L);
        uint32_t w = c / 64;
        uint64_t bit = 1ull << (c % 64);
        uint32_t j;
        if (n > 0 && words[n - 1] == w) {
            j = n - 1;
        } else if (n > 0 && words[0] == w) {
            j = 0;
        } else {
            j = n++;
            words[j] = w;
            masks[j] = 0;
        }
        masks[j] |= bit;
    }
    return n;
}

/* Make unavailable every placement of orientation o whose anchor is in rows
 * r0 .. r0+nrows-1 (mod L) and in the columns given by (words, masks). */
static void clear_block(sample_t *s, uint32_t o, uint32_t r0, uint32_t nrows,
                        const uint32_t *words, const uint64_t *masks, uint32_t nw)
{
    uint64_t L = s->L;
    for (uint32_t i = 0; i < nrows; ++i) {
        uint64_t y = ((uint64_t)r0 + i) % L;
        for (uint32_t j = 0; j < nw; ++j) {
            uint64_t *word = s->avail[o] + y * s->Wd + words[j];
            uint64_t hit = *word & masks[j];
            if (hit) {
                *word &= ~hit;
                int c = popcount64(hit);
                s->cnt[o * L + y] -= c;
                s->A -= (uint64_t)c;
                s->wchg += 1;
            }
        }
    }
}

/* Deposit of k-mer (o, y, x): every placement that covers one of its k sites
 * stops being available (Sec. II.B, "viable" placements).
 *   horizontal at (y,x): H anchors (y, x-k+1 .. x+k-1), V anchors
 *                        (y-k+1 .. y, x .. x+k-1);
 *   vertical at (y,x):   V anchors (y-k+1 .. y+k-1, x), H anchors
 *                        (y .. y+k-1, x-k+1 .. x).
 * Runs of 2k-1 that exceed L cover each residue once. */
static void clear_blocked(sample_t *s, uint32_t o, uint32_t y, uint32_t x,
                          uint32_t *words, uint64_t *masks)
{
    uint32_t L = s->L, k = s->k;
    uint32_t strip = (2 * k - 1 < L) ? 2 * k - 1 : L;
    uint32_t back = (uint32_t)mod_l((int64_t)x - (int64_t)k + 1, L);
    uint32_t up = (uint32_t)mod_l((int64_t)y - (int64_t)k + 1, L);
    uint32_t nw;
    if (o == 0) {
        nw = interval_masks(L, back, strip, words, masks);
        clear_block(s, 0, y, 1, words, masks, nw);
        nw = interval_masks(L, x, k, words, masks);
        clear_block(s, 1, up, k, words, masks, nw);
    } else {
        nw = interval_masks(L, x, 1, words, masks);
        clear_block(s, 1, up, strip, words, masks, nw);
        nw = interval_masks(L, back, k, words, masks);
        clear_block(s, 0, y, k, words, masks, nw);
    }
}

/* Merge the clusters of k-mers m and n, which touch through a contact whose
 * unwrapped vector anchor_m - anchor_n is (vx, vy).  The smaller cluster is
 * relabelled and its members' displacements are shifted so that
 * D_m - D_n = v afterwards (Sec. II.C, II.D). */
static void merge(sample_t *s, int64_t m, int64_t n, int64_t vx, int64_t vy)
{
    int64_t cm = s->cid[m], cn = s->cid[n];
    int64_t keep, gone, shx, shy;
    if (s->size[cn] <= s->size[cm]) {
        keep = cm; gone = cn;
        shx = (s->dx[m] - vx) - s->dx[n];
        shy = (s->dy[m] - vy) - s->dy[n];
    } else {
        keep = cn; gone = cm;
        shx = (s->dx[n] + vx) - s->dx[m];
        shy = (s->dy[n] + vy) - s->dy[m];
    }
    for (int64_t q = s->head[gone]; q >= 0; q = s->next[q]) {
        s->cid[q] = keep;
        s->dx[q] += shx;
        s->dy[q] += shy;
    }
    s->next[s->tail[keep]] = s->head[gone];
    s->tail[keep] = s->tail[gone];
    s->size[keep] += s->size[gone];
    s->wx[keep] |= s->wx[gone];
    s->wy[keep] |= s->wy[gone];
    s->head[gone] = -1;
    s->size[gone] = 0;
}

/* Nearest-neighbour contacts of the new k-mer m with occupied sites: for a
 * horizontal k-mer the left neighbour of site 0, the right neighbour of site
 * k-1 and the sites above and below every site; for a vertical one the
 * transpose.  Sites of m itself count (k = L, or L <= 2).  For each contact
 * the unwrapped vector v = anchor_m - anchor_n through it either merges two
 * clusters or, inside one cluster, closes a cycle whose winding is
 * w = D_m - D_n - v; a non-zero component of w is a wrap in that direction
 * (Sec. II.D, exact form of the paper's 2k test). */
static void contacts(sample_t *s, int64_t m, int *wrapx, int *wrapy)
{
    int64_t L = s->L, k = s->k;
    int64_t ax = s->anchor[m] % L, ay = s->anchor[m] / L;
    int64_t umx = s->orient[m] == 0 ? 1 : 0, umy = 1 - umx;
    static const int64_t ex[4] = {1, -1, 0, 0}, ey[4] = {0, 0, 1, -1};
    for (int64_t i = 0; i < k; ++i) {
        for (int dir = 0; dir < 4; ++dir) {
            int along = (ex[dir] == umx && ey[dir] == umy);
            int against = (ex[dir] == -umx && ey[dir] == -umy);
            if (along && i != k - 1) continue;
            if (against && i != 0) continue;
            int64_t bx = mod_l(ax + i * umx + ex[dir], L);
            int64_t by = mod_l(ay + i * umy + ey[dir], L);
            int64_t n = s->map[by * L + bx];
            if (n < 0) continue;
            int64_t nx = s->anchor[n] % L, ny = s->anchor[n] / L;
            int64_t unx = s->orient[n] == 0 ? 1 : 0, uny = 1 - unx;
            int64_t j = mod_l((bx - nx) * unx + (by - ny) * uny, L);
            int64_t vx = j * unx - i * umx - ex[dir];
            int64_t vy = j * uny - i * umy - ey[dir];
            if (s->cid[n] != s->cid[m]) {
                merge(s, m, n, vx, vy);
            } else {
                int64_t wx = s->dx[m] - s->dx[n] - vx;
                int64_t wy = s->dy[m] - s->dy[n] - vy;
                if (wx != 0) {
                    s->wx[s->cid[m]] = 1;
                    *wrapx = 1;
                }
                if (wy != 0) {
                    s->wy[s->cid[m]] = 1;
                    *wrapy = 1;
                }
            }
        }
    }
}

/* Cluster sizes in sites, histogrammed into hist[0..cap-1]. */
static void cluster_histogram(const sample_t *s, uint64_t nkmers, uint64_t *hist, uint64_t cap)
{
    for (uint64_t c = 0; c < cap; ++c) hist[c] = 0;
    for (uint64_t c = 0; c < nkmers; ++c) {
        if (s->head[c] < 0) continue;
        uint64_t sites = (uint64_t)s->size[c] * s->k;
        if (sites < cap) hist[sites] += 1;
    }
}

/* End-of-run checks.  Jamming means no row and no column holds k empty sites
 * in a row (cyclically), the availability bits and counts are all zero, every
 * cluster wraps (Appendix A, Proposition), and percolation happened no later
 * than jamming (Appendix A, Consequence). */
static int check_jammed(const sample_t *s, int64_t nkmers, const rsao_result_t *r, int h_only)
{
    uint64_t L = s->L, k = s->k;
    for (int o = 0; o < (h_only ? 1 : 2); ++o) {
        for (uint64_t line = 0; line < L; ++line) {
            /* longest cyclic run of empty sites along this row (o=0) or column */
            uint64_t run = 0, best = 0, first_run = 0, all_empty = 1;
            for (uint64_t i = 0; i < L; ++i) {
                uint64_t site = o == 0 ? line * L + i : i * L + line;
                if (s->map[site] < 0) {
                    ++run;
                    if (run > best) best = run;
                } else {
                    if (all_empty) first_run = run;
                    all_empty = 0;
                    run = 0;
                }
            }
            if (all_empty) return RSAO_ESCAN;
            if (run + first_run > best) best = run + first_run; /* joins across the seam */
            if (best >= k) return RSAO_ESCAN;
        }
    }
    for (int o = 0; o < 2; ++o) {
        for (uint64_t i = 0; i < L * s->Wd; ++i)
            if (s->avail[o][i]) return RSAO_ECOUNT;
        for (uint64_t y = 0; y < L; ++y)
            if (s->cnt[o * L + y] != 0) return RSAO_ECOUNT;
    }
    if (s->A != 0) return RSAO_ECOUNT;
    for (int64_t c = 0; c < nkmers; ++c)
        if (s->head[c] >= 0 && !s->wx[c] && !s->wy[c]) return RSAO_ENOWRAP;
    if (r->n_wrap_any < 1 || r->n_wrap_any > r->n_jam) return RSAO_EORDER;
    return RSAO_OK;
}

static int valid_desc(const rsao_desc_t *d)
{
    return d && d->k >= 1 && d->k <= d->L && d->L <= 32768 && (d->flags & ~(RSAO_FLAG_H_ONLY | RSAO_FLAG_TRACK_CLUSTERS | RSAO_FLAG_CONTACTS)) == 0;
}

/* One run, with optional extras for the contact census (out3 != NULL). */
static int run_sample(const rsao_desc_t *d, rsao_result_t *r, uint32_t *seq, uint64_t seq_cap,
                      int64_t snap_step, uint64_t *snap_hist, uint64_t snap_cap, uint64_t *out3)
{
    memset(r, 0, sizeof(*r));
    r->n_jam = r->n_wrap_x = r->n_wrap_y = r->n_wrap_any = -1;
    r->n_clusters_jam = r->n_nonwrapping_jam = -1;
    if (!valid_desc(d)) return r->status = RSAO_EINVAL;
    sample_t s;
    int rc = init_sample(&s, d);
    if (rc) return r->status = rc;
    uint64_t L = d->L, k = d->k;
    uint32_t *words = (uint32_t *)malloc((s.Wd + 1) * sizeof(uint32_t));
    uint64_t *masks = (uint64_t *)malloc((s.Wd + 1) * sizeof(uint64_t));
    if (!words || !masks) {
        free(words); free(masks); free_sample(&s);
        return r->status = RSAO_ENOMEM;
    }
    uint64_t A0 = s.A;
    uint32_t key[2] = {(uint32_t)d->seed, (uint32_t)(d->seed >> 32)};
    int wrapx = 0, wrapy = 0;
    uint64_t t = 0;
    uint64_t seq_hash = 0;
    int status = RSAO_OK;
    while (s.A > 0) {
        /* draw (Sec. II.B: a uniformly random viable placement) */
        uint32_t ctr[4] = {(uint32_t)t, d->sample, 0, 0}, rnd[4];
        rsao_philox4x32_10(ctr, key, rnd);
        uint64_t u = (uint64_t)rnd[0] | ((uint64_t)rnd[1] << 32);
        uint32_t rank = rsao_rank(u, (uint32_t)s.A);
        uint32_t P = select_placement(&s, rank);
        uint32_t o = (uint32_t)(P / (L * L));
        uint32_t y = (uint32_t)((P % (L * L)) / L), x = (uint32_t)(P % L);
        if (seq) {
            if (t >= seq_cap) {
                status = RSAO_ECAPACITY;
                break;
            }
            seq[t] = P;
        }
        seq_hash += rsao_mix64((t << 32) | P);
        /* deposit */
        clear_blocked(&s, o, y, x, words, masks);
        for (uint64_t i = 0; i < k; ++i) {
            uint64_t sx = o == 0 ? (x + i) % L : x;
            uint64_t sy = o == 0 ? y : (y + i) % L;
            s.map[sy * L + sx] = (int32_t)t;
        }
        s.anchor[t] = y * (uint32_t)L + x;
        s.orient[t] = (uint8_t)o;
        s.cid[t] = (int64_t)t;
        s.dx[t] = s.dy[t] = 0;
        s.next[t] = -1;
        s.head[t] = s.tail[t] = (int64_t)t;
        s.size[t] = 1;
        s.wx[t] = s.wy[t] = 0;
        /* cluster labelling and wrap check (Sec. II.C, II.D) */
        contacts(&s, (int64_t)t, &wrapx, &wrapy);
        if (wrapx && r->n_wrap_x < 0) r->n_wrap_x = (int64_t)t + 1;
        if (wrapy && r->n_wrap_y < 0) r->n_wrap_y = (int64_t)t + 1;
        ++t;
        if (snap_hist && snap_step > 0 && (int64_t)t == snap_step)
            cluster_histogram(&s, t, snap_hist, snap_cap);
    }
    r->n_jam = (int64_t)t;
    if (r->n_wrap_x > 0) r->n_wrap_any = r->n_wrap_x;
    if (r->n_wrap_y > 0 && (r->n_wrap_any < 0 || r->n_wrap_y < r->n_wrap_any))
        r->n_wrap_any = r->n_wrap_y;
    r->seq_hash = seq_hash;
    uint64_t occ = 0;
    for (uint64_t site = 0; site < L * L; ++site)
        if (s.map[site] >= 0) occ += rsao_mix64((site << 32) | (uint32_t)s.map[site]);
    r->occ_hash = occ;
    int32_t nclusters = 0, nonwrap = 0;
    for (uint64_t c = 0; c < t; ++c) {
        if (s.head[c] < 0) continue;
        ++nclusters;
        if (!s.wx[c] && !s.wy[c]) ++nonwrap;
    }
    r->n_clusters_jam = nclusters;
    r->n_nonwrapping_jam = nonwrap;
    /* Algorithmic-byte model: initialise the site map (4 B/site) and both
     * availability bitmaps; per deposit write k map entries, read the 2k+2
     * neighbour entries, read one bitmap row for the select and write one
     * 16 B k-mer record; read and write back every availability word whose
     * value changes. */
    r->wchg_words = s.wchg;
    r->alg_bytes = 4 * L * L + 16 * L * s.Wd + t * (4 * k + 4 * (2 * k + 2) + 8 * s.Wd + 16) +
                   16 * s.wchg;
    if (status == RSAO_OK && A0 != 0) status = check_jammed(&s, (int64_t)t, r, d->flags & 1);
    if (out3 && status == RSAO_OK) {
        /* contact census at jamming: each unordered nearest-neighbour pair of
         * occupied sites in different k-mers, counted once (right and down
         * neighbour of every site; on L <= 2 a pair can be met twice and is
         * then counted twice, as the lattice has two bonds between them). */
        out3[0] = out3[1] = out3[2] = 0;
        for (uint64_t yy = 0; yy < L; ++yy) {
            for (uint64_t xx = 0; xx < L; ++xx) {
                int32_t a = s.map[yy * L + xx];
                if (a < 0) continue;
                uint64_t nb[2] = {yy * L + (xx + 1) % L, ((yy + 1) % L) * L + xx};
                for (int q = 0; q < 2; ++q) {
                    int32_t b = s.map[nb[q]];
                    if (b < 0 || b == a) continue;
                    int oa = s.orient[a], ob = s.orient[b];
                    if (oa != ob) out3[2] += 1;
                    else out3[oa] += 1;
                }
            }
        }
    }
    free(words);
    free(masks);
    free_sample(&s);
    return r->status = status;
}

int rsao_run(const rsao_desc_t *d, rsao_result_t *r, uint32_t *seq, uint64_t seq_cap,
             int64_t snap_step, uint64_t *snap_hist, uint64_t snap_cap)
{
    return run_sample(d, r, seq, seq_cap, snap_step, snap_hist, snap_cap, NULL);
}

int rsao_run_many(const rsao_desc_t *d, rsao_result_t *r, uint32_t n)
{
    int worst = RSAO_OK;
    for (uint32_t i = 0; i < n; ++i) {
        int rc = run_sample(&d[i], &r[i], NULL, 0, 0, NULL, 0, NULL);
        if (rc < worst) worst = rc;
    }
    return worst;
}

int rsao_contacts_at_jamming(const rsao_desc_t *d, uint64_t out3[3])
{
    rsao_result_t r;
    return run_sample(d, &r, NULL, 0, 0, NULL, 0, out3);
}
