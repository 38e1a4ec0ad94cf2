// rsa_kernels.hip -- gfx950 kernels for random sequential adsorption of linear
// k-mers on an L x L torus, run to jamming with first-wrap tracking
// (Slutskii, Barash, Tarasevich, arXiv:1810.06800).
//
// One workgroup runs one sample at a time and pulls the next sample from a
// device work queue when it is done (persistent form).  Its waves split the
// method in two decoupled chains:
//
//  * the selecting waves (wave 0, helped by NSEL-1 more) run the deposition
//    of Sec. II.B without rejected attempts: per step they draw a rank
//    uniformly among the A_t available placements (Philox4x32-10 keyed by the
//    seed, counter (t, sample, 0, 0)), find that placement by hierarchical
//    wavefront prefix sums over per-row counts held in LDS and one bitmap row
//    read from HBM, and clear every placement the new k-mer blocks with
//    coalesced word read-modify-writes, decrementing the counts;
//  * the labelling wave (the last wave) follows behind through an LDS ring of
//    placements, writes the site map and runs union-find over k-mer ids with
//    unwrapped displacement vectors (Sec. II.C-II.E).  A contact that closes a
//    cycle inside one cluster has winding w = D_m - D_n - v; a non-zero
//    component is a wrap in that direction (Sec. II.D; the exact form of the
//    paper's 2k test).  It takes up to 64 deposits at once, resolves the
//    clusters they touch with parallel finds, and merges them in deposit
//    order in an LDS-resident union-find, so the first wrap step is exact.
//
// The two chains share only the ring, so the union-find latency stays off the
// select/clear critical path.  Nothing here uses MFMA: the work is integer
// bitmap and graph work bound by memory latency and bandwidth.
#include <hip/hip_runtime.h>

#include "rsa_device.h"

namespace rsa {

constexpr uint32_t kUnroll = 4;   // independent bitmap words in flight per lane

// Internal failure codes reported in the result's status field.  They mean a
// broken invariant (counts that disagree with the bitmaps, a cycle in the
// union-find); the sample then stops instead of reading out of bounds.
constexpr int32_t kErrSelect = -100;
constexpr int32_t kErrLabel = -101;
constexpr uint32_t kMaxHops = 64;   // union by rank keeps trees below log2(L^2) levels

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// LDS-only hand-offs between waves of one workgroup: LDS instructions of a
// wave execute in issue order, so a compiler-only fence is enough to order a
// payload before (after) the flag that publishes (consumes) it.
__device__ __forceinline__ uint32_t lds_load(const uint32_t *p)
{
    uint32_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return v;
}

__device__ __forceinline__ void lds_store(uint32_t *p, uint32_t v)
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lds_peek(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t wave_scan(uint32_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v)
{
#pragma unroll
    for (uint32_t d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v)
{
#pragma unroll
    for (uint32_t d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ uint32_t first_lane(uint64_t ballot) { return (uint32_t)(__ffsll((long long)ballot) - 1); }

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, key bumped by
// the Weyl constants between rounds.  Only output words 0 and 1 are used.
__device__ __forceinline__ uint64_t philox_u64(uint32_t c0, uint32_t c1, uint32_t k0, uint32_t k1)
{
    uint32_t c2 = 0, c3 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return (uint64_t)c0 | ((uint64_t)c1 << 32);
}

// floor(u * a / 2^64) from two 32x32 products.
__device__ __forceinline__ uint32_t draw_rank(uint64_t u, uint32_t a)
{
    uint64_t lo = (uint64_t)(uint32_t)u * a;
    uint64_t hi = (u >> 32) * (uint64_t)a;
    return (uint32_t)((hi + (lo >> 32)) >> 32);
}

// SplitMix64 finalizer (Steele, Lea, Flood, OOPSLA'14).
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Per-workgroup view of one sample
// ---------------------------------------------------------------------------

struct Hdr {
    uint32_t sel_progress;   // placements published in the ring
    uint32_t sel_done;       // 1 + n_jam once selection has finished, else 0
    uint32_t lab_progress;   // ring entries the labelling wave has taken
    uint32_t lab_exit;       // labelling wave finished
    uint32_t clr_gen;        // clear requests published to helper waves
    uint32_t clr_done;       // helper completions, cumulative
    uint32_t cur_p;          // placement being cleared
    uint32_t sample;         // descriptor index of the current sample
    uint32_t nslots;         // labelling: local union-find slots in use
    int32_t nx, ny;          // first wrap steps (1-based) or -1
    uint32_t nclusters, nonwrap;
    int32_t status;          // 0, or kErrSelect / kErrLabel
    uint32_t pad[2];
    unsigned long long wchg;
    unsigned long long occ;
    unsigned long long seqh;
};

struct Ctx {
    uint32_t L, k, wd, flags, sample, L2;
    uint32_t ncap;     // k-mer records in the slab, L*L/k + 1
    uint32_t k0, k1;   // Philox key
    FastDiv fL, fk, fC;
    uint64_t *av[2];
    int32_t *map;
    int4 *node;
    uint32_t *kmer;
    Hdr *h;
    uint32_t *cnt0, *cnt1, *cnt2;
    uint32_t n1, n2;
    uint32_t *ring, *banc;
    uint32_t *e_step, *e_ms;
    int32_t *e_vx, *e_vy;
    uint32_t *s_par, *s_meta, *s_gid;
    int32_t *s_dx, *s_dy;
    uint32_t *h_key, *h_val;
};

__device__ __forceinline__ uint32_t row_count(const Ctx &c, uint32_t r)
{
    return (lds_peek(&c.cnt0[r >> 1]) >> ((r & 1) << 4)) & 0xFFFFu;
}

__device__ __forceinline__ void count_sub(const Ctx &c, uint32_t r, uint32_t n)
{
    atomicSub(&c.cnt0[r >> 1], n << ((r & 1) << 4));
    atomicSub(&c.cnt1[r >> 6], n);
    atomicSub(&c.cnt2[r >> 12], n);
}

// Bits of word w inside [lo, hi) (column indices).
__device__ __forceinline__ uint64_t piece_mask(uint32_t lo, uint32_t hi, uint32_t w)
{
    uint32_t b0 = w * 64, b1 = b0 + 64;
    uint32_t a = lo > b0 ? lo : b0;
    uint32_t b = hi < b1 ? hi : b1;
    if (a >= b) return 0;
    uint32_t s = a - b0, e = b - b0;
    uint64_t upto = e == 64 ? ~0ull : ((1ull << e) - 1);
    return upto & ~((1ull << s) - 1);
}

// Bits of word w inside the cyclic column interval [c0, c0 + len) mod L.
__device__ __forceinline__ uint64_t col_mask(uint32_t L, uint32_t c0, uint32_t len, uint32_t w)
{
    if (len >= L) return piece_mask(0, L, w);
    uint32_t end = c0 + len;
    uint64_t m = piece_mask(c0, end < L ? end : L, w);
    if (end > L) m |= piece_mask(0, end - L, w);
    return m;
}

// Make unavailable every placement of orientation o anchored in rows
// row0 .. row0+nrows-1 (mod L) and in the cyclic columns [c0, c0+len).
// Wave `wv` of `nwv` takes its share; each lane holds kUnroll words in flight.
__device__ void clear_region(const Ctx &c, uint32_t o, uint32_t row0, uint32_t nrows, uint32_t c0,
                             uint32_t len, uint32_t wv, uint32_t nwv, uint32_t &wchg)
{
    const uint32_t lane = lane_id(), L = c.L, wd = c.wd;
    // words the column interval touches, each once: the piece [c0, ...) from
    // word a0, then (after the seam) words 0 .. nB-1 below a0
    uint32_t a0, nA, nB;
    if (len >= L) {
        a0 = 0;
        nA = wd;
        nB = 0;
    } else {
        uint32_t end = c0 + len;
        uint32_t endA = end < L ? end : L;
        a0 = c0 >> 6;
        nA = ((endA - 1) >> 6) - a0 + 1;
        nB = 0;
        if (end > L) {
            uint32_t b1 = (end - L - 1) >> 6;
            nB = (b1 == a0) ? b1 : b1 + 1;
        }
    }
    const uint32_t nw = nA + nB;
    uint64_t *base = c.av[o];
    const uint32_t rowbase = o * L;
    if (nw <= 64) {
        uint32_t lg = nw <= 1 ? 0 : 32 - __clz(nw - 1);
        uint32_t rows_per = 64u >> lg;
        uint32_t wsub = lane & ((1u << lg) - 1), rsub = lane >> lg;
        bool wact = wsub < nw;
        uint32_t w = wsub < nA ? a0 + wsub : wsub - nA;
        uint64_t mask = wact ? col_mask(L, c0, len, w) : 0;
        uint32_t stride = rows_per * nwv;
        for (uint32_t rb = wv * rows_per; rb < nrows; rb += stride * kUnroll) {
            uint64_t old[kUnroll];
            uint32_t row[kUnroll];
            bool act[kUnroll];
#pragma unroll
            for (uint32_t u = 0; u < kUnroll; ++u) {
                uint32_t i = rb + u * stride + rsub;
                act[u] = wact && i < nrows;
                uint32_t r = row0 + i;
                r = r >= L ? r - L : r;
                row[u] = r;
                old[u] = act[u] ? base[(size_t)r * wd + w] : 0;
            }
#pragma unroll
            for (uint32_t u = 0; u < kUnroll; ++u) {
                uint64_t hit = old[u] & mask;
                if (hit) {
                    base[(size_t)row[u] * wd + w] = old[u] & ~hit;
                    count_sub(c, rowbase + row[u], (uint32_t)__popcll(hit));
                    ++wchg;
                }
            }
        }
    } else {
        for (uint32_t i = wv; i < nrows; i += nwv) {
            uint32_t r = row0 + i;
            r = r >= L ? r - L : r;
            uint64_t *rowp = base + (size_t)r * wd;
            uint32_t cleared = 0;
            for (uint32_t j0 = 0; j0 < nw; j0 += 64 * kUnroll) {
                uint64_t old[kUnroll], mask[kUnroll];
                uint32_t w[kUnroll];
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u) {
                    uint32_t j = j0 + u * 64 + lane;
                    bool act = j < nw;
                    w[u] = j < nA ? a0 + j : j - nA;
                    mask[u] = act ? col_mask(L, c0, len, w[u]) : 0;
                    old[u] = act ? rowp[w[u]] : 0;
                }
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u) {
                    uint64_t hit = old[u] & mask[u];
                    if (hit) {
                        rowp[w[u]] = old[u] & ~hit;
                        cleared += (uint32_t)__popcll(hit);
                        ++wchg;
                    }
                }
            }
            uint32_t tot = wave_sum32(cleared);
            if (lane == 0 && tot) count_sub(c, rowbase + r, tot);
        }
    }
}

// Deposit of k-mer (o, y, x): every placement covering one of its sites stops
// being available (Sec. II.B).  Horizontal at (y, x): H anchors in row y,
// columns x-k+1 .. x+k-1, and V anchors in rows y-k+1 .. y, columns
// x .. x+k-1.  Vertical: the transpose.  Runs longer than L wrap once.
__device__ void clear_blocked(const Ctx &c, uint32_t o, uint32_t y, uint32_t x, uint32_t wv,
                              uint32_t nwv, uint32_t &wchg)
{
    const uint32_t L = c.L, k = c.k;
    uint32_t strip = 2 * k - 1 < L ? 2 * k - 1 : L;
    uint32_t back = x + L - (k - 1);
    back = back >= L ? back - L : back;
    uint32_t up = y + L - (k - 1);
    up = up >= L ? up - L : up;
    if (o == 0) {
        clear_region(c, 0, y, 1, back, strip, wv, nwv, wchg);
        clear_region(c, 1, up, k, x, k, wv, nwv, wchg);
    } else {
        clear_region(c, 1, up, strip, x, 1, wv, nwv, wchg);
        clear_region(c, 0, y, k, back, k, wv, nwv, wchg);
    }
}

// ---------------------------------------------------------------------------
// Selecting wave
// ---------------------------------------------------------------------------

template <int NSEL>
__device__ void selector(Ctx &c)
{
    const uint32_t lane = lane_id();
    const uint32_t L = c.L, k = c.k, rows = 2 * L;
    uint64_t occ = 0, seqh = 0;
    uint32_t wchg = 0;
    uint64_t u_pre = 0;
    uint32_t t = 0;
    for (;; ++t) {
        // the labelling wave must have taken ring slot t before it is reused
        if (t >= kRing) {
            while (!lds_load(&c.h->lab_exit) && t - lds_load(&c.h->lab_progress) >= kRing)
                __builtin_amdgcn_s_sleep(2);
        }
        // level 2 (4096-row sums) also gives A_t
        uint32_t v = lane < c.n2 ? lds_peek(&c.cnt2[lane]) : 0;
        uint32_t inc = wave_scan(v);
        uint32_t A = __shfl(inc, 63, 64);
        if (A == 0) break;
        if ((t & 63) == 0) u_pre = philox_u64(t + lane, c.sample, c.k0, c.k1);
        uint64_t u = __shfl(u_pre, t & 63, 64);
        uint32_t r = draw_rank(u, A);
        uint64_t bal = __ballot(inc > r);
        if (bal == 0) {   // cannot happen with consistent counts
            if (lane == 0) c.h->status = kErrSelect;
            break;
        }
        uint32_t g = first_lane(bal);
        r -= __shfl(inc - v, g, 64);
        // level 1 (64-row sums)
        uint32_t i1 = g * 64 + lane;
        v = i1 < c.n1 ? lds_peek(&c.cnt1[i1]) : 0;
        inc = wave_scan(v);
        bal = __ballot(inc > r);
        if (bal == 0) {
            if (lane == 0) c.h->status = kErrSelect;
            break;
        }
        uint32_t l1 = first_lane(bal);
        r -= __shfl(inc - v, l1, 64);
        g = g * 64 + l1;
        // level 0 (rows)
        uint32_t i0 = g * 64 + lane;
        v = i0 < rows ? row_count(c, i0) : 0;
        inc = wave_scan(v);
        bal = __ballot(inc > r);
        if (bal == 0) {
            if (lane == 0) c.h->status = kErrSelect;
            break;
        }
        uint32_t l0 = first_lane(bal);
        r -= __shfl(inc - v, l0, 64);
        const uint32_t R = g * 64 + l0;
        const uint32_t o = R >= L ? 1u : 0u;
        const uint32_t y = R - o * L;
        // the chosen row: lane holds words lane, lane+64, ...
        const uint64_t *rowp = c.av[o] + (size_t)y * c.wd;
        const uint32_t per = (c.wd + 63) >> 6;
        uint64_t w[8];
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
            uint32_t wi = lane + 64 * j;
            w[j] = (j < per && wi < c.wd) ? rowp[wi] : 0;
        }
        uint64_t word = 0;
        uint32_t wsel = 0;
        bool found = false;
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
            if (j < per) {
                uint32_t pc = (uint32_t)__popcll(w[j]);
                uint32_t pinc = wave_scan(pc);
                uint32_t tot = __shfl(pinc, 63, 64);
                if (r < tot) {
                    uint32_t l = first_lane(__ballot(pinc > r));
                    r -= __shfl(pinc - pc, l, 64);
                    word = __shfl(w[j], l, 64);
                    wsel = l + 64 * j;
                    found = true;
                    break;
                }
                r -= tot;
            }
        }
        // r-th set bit of the word
        uint32_t below = (uint32_t)__popcll(word & ((1ull << lane) - 1));
        bal = __ballot(((word >> lane) & 1) && below == r);
        if (!found || bal == 0 || R >= rows) {
            if (lane == 0) c.h->status = kErrSelect;
            break;
        }
        const uint32_t x = wsel * 64 + first_lane(bal);
        if (x >= L) {
            if (lane == 0) c.h->status = kErrSelect;
            break;
        }
        const uint32_t P = o * c.L2 + y * L + x;
        // hand the placement to the labelling wave
        if (lane == 0) {
            c.ring[t & (kRing - 1)] = P;
            lds_store(&c.h->sel_progress, t + 1);
        }
        seqh += mix64(((uint64_t)t << 32) | P);
        for (uint32_t i = lane; i < k; i += 64) {
            uint32_t s;
            if (o == 0) {
                uint32_t xx = x + i;
                xx = xx >= L ? xx - L : xx;
                s = y * L + xx;
            } else {
                uint32_t yy = y + i;
                yy = yy >= L ? yy - L : yy;
                s = yy * L + x;
            }
            occ += mix64(((uint64_t)s << 32) | t);
        }
        if (NSEL > 1) {
            if (lane == 0) {
                c.h->cur_p = P;
                lds_store(&c.h->clr_gen, t + 1);
            }
        }
        clear_blocked(c, o, y, x, 0, NSEL, wchg);
        if (NSEL > 1) {
            // helpers' bitmap stores must be visible before the next select
            uint32_t want = (t + 1) * (NSEL - 1);
            while (lds_load(&c.h->clr_done) < want) __builtin_amdgcn_s_sleep(1);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
    }
    occ = wave_sum64(occ);
    uint32_t wsum = wave_sum32(wchg);
    if (lane == 0) {
        atomicAdd(&c.h->occ, (unsigned long long)occ);
        atomicAdd(&c.h->wchg, (unsigned long long)wsum);
        c.h->seqh = seqh;
        lds_store(&c.h->sel_done, t + 1);
    }
}

template <int NSEL>
__device__ void helper(Ctx &c, uint32_t wv)
{
    const uint32_t lane = lane_id();
    uint32_t wchg = 0;
    uint32_t g = 0;
    for (;;) {
        uint32_t gen;
        bool stop = false;
        for (;;) {
            gen = lds_load(&c.h->clr_gen);
            if (gen > g) break;
            if (lds_load(&c.h->sel_done)) {
                stop = true;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (stop) break;
        g = gen;
        uint32_t P = lds_peek(&c.h->cur_p);
        uint32_t o = P >= c.L2 ? 1u : 0u;
        uint32_t rem = P - o * c.L2;
        uint32_t y = fdiv(rem, c.fL);
        uint32_t x = rem - y * c.L;
        clear_blocked(c, o, y, x, wv, NSEL, wchg);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) atomicAdd(&c.h->clr_done, 1u);
    }
    uint32_t wsum = wave_sum32(wchg);
    if (lane == 0) atomicAdd(&c.h->wchg, (unsigned long long)wsum);
}

// ---------------------------------------------------------------------------
// Labelling wave: site map, contacts, union-find with displacements
// ---------------------------------------------------------------------------

// Root of global k-mer x and x's displacement from it (read-only walk).
__device__ __forceinline__ bool global_find(const Ctx &c, uint32_t x, uint32_t &root, int32_t &dx,
                                            int32_t &dy, uint32_t &meta)
{
    uint32_t cur = x;
    int32_t ax = 0, ay = 0;
    int4 nd = make_int4(0, 0, 0, 0);
    bool ok = false;
    for (uint32_t hop = 0; hop < kMaxHops; ++hop) {
        nd = c.node[cur];
        if ((uint32_t)nd.x == cur) {
            ok = true;
            break;
        }
        if ((uint32_t)nd.x >= c.ncap) break;   // not a k-mer id: corrupted record
        ax += nd.y;
        ay += nd.z;
        cur = (uint32_t)nd.x;
    }
    root = cur;
    dx = ax;
    dy = ay;
    meta = (uint32_t)nd.w;
    return ok;
}

// Local union-find over LDS slots, path halving with displacements.
__device__ __forceinline__ uint32_t local_find(const Ctx &c, uint32_t a, int32_t &dx, int32_t &dy)
{
    uint32_t x = a;
    int32_t ax = 0, ay = 0;
    for (uint32_t it = 0; it < kSlots; ++it) {
        uint32_t p = c.s_par[x];
        if (p == x) break;
        uint32_t gp = c.s_par[p];
        if (gp == p) {
            ax += c.s_dx[x];
            ay += c.s_dy[x];
            x = p;
            break;
        }
        int32_t hx = c.s_dx[x] + c.s_dx[p], hy = c.s_dy[x] + c.s_dy[p];
        c.s_par[x] = gp;
        c.s_dx[x] = hx;
        c.s_dy[x] = hy;
        ax += hx;
        ay += hy;
        x = gp;
    }
    dx = ax;
    dy = ay;
    return x;
}

struct LabelState {
    uint32_t base;   // k-mers base .. base+nb-1 own slots 0 .. nb-1
    uint32_t nb;
    int32_t nx, ny;
};

__device__ void reset_slots(const Ctx &c, const LabelState &ls)
{
    const uint32_t lane = lane_id();
    for (uint32_t s = lane; s < ls.nb; s += 64) {
        c.s_par[s] = s;
        c.s_dx[s] = 0;
        c.s_dy[s] = 0;
        c.s_meta[s] = 0;
        c.s_gid[s] = ls.base + s;
    }
    for (uint32_t i = lane; i < kHash; i += 64) c.h_key[i] = 0;
    if (lane == 0) c.h->nslots = ls.nb;
}

// Write the local forest back into the global one.
__device__ void write_back(const Ctx &c)
{
    const uint32_t lane = lane_id();
    const uint32_t ns = c.h->nslots;
    for (uint32_t s = lane; s < ns; s += 64) {
        uint32_t x = s;
        int32_t dx = 0, dy = 0;
        for (uint32_t it = 0; it < kSlots && c.s_par[x] != x; ++it) {
            dx += c.s_dx[x];
            dy += c.s_dy[x];
            x = c.s_par[x];
        }
        uint32_t g = c.s_gid[s];
        if (x == s)
            c.node[g] = make_int4((int)g, 0, 0, (int)c.s_meta[s]);
        else
            c.node[g] = make_int4((int)c.s_gid[x], dx, dy, 0);
    }
}

// Slot of the global k-mer id (a batch k-mer, or the root of an older one).
// All lanes of the wave call this together; `need` marks lanes with an id.
__device__ __forceinline__ uint32_t resolve_slot(const Ctx &c, const LabelState &ls, bool need,
                                                 uint32_t id, int32_t &dx, int32_t &dy)
{
    dx = 0;
    dy = 0;
    bool local = need && id >= ls.base;
    bool global = need && !local;
    uint32_t root = 0, meta = 0;
    if (global) {
        if (!global_find(c, id, root, dx, dy, meta)) {
            c.h->status = kErrLabel;
            global = false;
        } else if (root != id) {
            // shortcut the walked path for later finds: id now points at its root
            c.node[id] = make_int4((int)root, dx, dy, 0);
        }
    }
    // claim a hash entry for the root
    uint32_t pos = 0;
    bool won = false;
    if (global) {
        uint32_t hsh = (root * 0x9E3779B1u) >> 22;   // kHash = 1024
        for (uint32_t probe = 0; probe < kHash; ++probe) {
            uint32_t prev = atomicCAS(&c.h_key[hsh], 0u, root + 1);
            if (prev == 0) {
                won = true;
                break;
            }
            if (prev == root + 1) break;
            hsh = (hsh + 1) & (kHash - 1);
        }
        pos = hsh;
    }
    if (won) {
        uint32_t s = atomicAdd(&c.h->nslots, 1u);
        c.s_par[s] = s;
        c.s_dx[s] = 0;
        c.s_dy[s] = 0;
        c.s_meta[s] = meta;
        c.s_gid[s] = root;
        c.h_val[pos] = s;
    }
    __builtin_amdgcn_wave_barrier();
    uint32_t slot = 0;
    if (local) slot = id - ls.base;
    if (global) slot = c.h_val[pos];
    return slot;
}

// Resolve the chunk's edges to slots, then merge in deposit order.
__device__ void process_chunk(const Ctx &c, LabelState &ls, uint32_t ne)
{
    const uint32_t lane = lane_id();
    if (ne == 0) return;
    // every edge can bring two new roots; make room first
    if (c.h->nslots + 2 * ne > kSlots) {
        write_back(c);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        uint32_t m_first = c.e_step[0];
        uint32_t end = ls.base + ls.nb;
        ls.base = m_first + 1;
        ls.nb = end - ls.base;
        reset_slots(c, ls);
        __builtin_amdgcn_wave_barrier();
    }
    for (uint32_t e0 = 0; e0 < ne; e0 += 64) {
        uint32_t e = e0 + lane;
        bool act = e < ne;
        uint32_t m = act ? c.e_step[e] : 0;
        uint32_t n = act ? c.e_ms[e] : 0;
        int32_t dmx, dmy, dnx, dny;
        uint32_t sm = resolve_slot(c, ls, act, m, dmx, dmy);
        uint32_t sn = resolve_slot(c, ls, act, n, dnx, dny);
        if (act) {
            c.e_ms[e] = sm | (sn << 16);
            c.e_vx[e] += dnx - dmx;
            c.e_vy[e] += dny - dmy;
        }
    }
    __builtin_amdgcn_wave_barrier();
    // merge in deposit order (every lane walks the same list)
    int32_t nx = ls.nx, ny = ls.ny;
    for (uint32_t e = 0; e < ne; ++e) {
        uint32_t ms = c.e_ms[e];
        int32_t vx = c.e_vx[e], vy = c.e_vy[e];
        int32_t dax, day, dbx, dby;
        uint32_t ra = local_find(c, ms & 0xFFFFu, dax, day);
        uint32_t rb = local_find(c, ms >> 16, dbx, dby);
        if (ra != rb) {
            uint32_t ma = c.s_meta[ra], mb = c.s_meta[rb];
            if ((ma & 0xFFu) < (mb & 0xFFu)) {
                c.s_par[ra] = rb;
                c.s_dx[ra] = vx - dax + dbx;
                c.s_dy[ra] = vy - day + dby;
                c.s_meta[rb] = mb | (ma & 0x300u);
            } else {
                c.s_par[rb] = ra;
                c.s_dx[rb] = dax - dbx - vx;
                c.s_dy[rb] = day - dby - vy;
                uint32_t bump = (ma & 0xFFu) == (mb & 0xFFu) ? 1u : 0u;
                c.s_meta[ra] = (ma | (mb & 0x300u)) + bump;
            }
        } else {
            int32_t wx = dax - dbx - vx, wy = day - dby - vy;
            if (wx != 0 || wy != 0) {
                uint32_t step = c.e_step[e];
                c.s_meta[ra] |= (wx != 0 ? 0x100u : 0u) | (wy != 0 ? 0x200u : 0u);
                if (wx != 0 && nx < 0) nx = (int32_t)step + 1;
                if (wy != 0 && ny < 0) ny = (int32_t)step + 1;
            }
        }
    }
    ls.nx = nx;
    ls.ny = ny;
    __builtin_amdgcn_wave_barrier();
}

__device__ void labeler(Ctx &c, bool track)
{
    const uint32_t lane = lane_id();
    const uint32_t L = c.L, k = c.k, nC = 2 * k + 2;
    const FastDiv fC = c.fC;
    LabelState ls;
    ls.nx = -1;
    ls.ny = -1;
    uint32_t tl = 0;
    for (;;) {
        uint32_t sp;
        bool finished = false;
        for (;;) {
            sp = lds_load(&c.h->sel_progress);
            if (sp > tl) break;
            uint32_t sd = lds_load(&c.h->sel_done);
            if (sd && tl + 1 >= sd) {
                finished = true;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (finished) break;
        const uint32_t B = sp - tl < kBatch ? sp - tl : kBatch;
        const uint32_t t1 = tl + B;
        // take the placements out of the ring
        if (lane < B) {
            uint32_t P = c.ring[(tl + lane) & (kRing - 1)];
            uint32_t o = P >= c.L2 ? 1u : 0u;
            uint32_t a = (P - o * c.L2) | (o << 31);
            c.banc[lane] = a;
            c.kmer[tl + lane] = a;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) lds_store(&c.h->lab_progress, t1);
        // site map of the batch
        for (uint32_t q = lane; q < B * k; q += 64) {
            uint32_t i = fdiv(q, c.fk);
            uint32_t s = q - i * k;
            uint32_t a = c.banc[i];
            uint32_t site = a & 0x7FFFFFFFu;
            uint32_t ay = fdiv(site, c.fL), ax = site - ay * L;
            if (a >> 31) {
                uint32_t yy = ay + s;
                yy = yy >= L ? yy - L : yy;
                site = yy * L + ax;
            } else {
                uint32_t xx = ax + s;
                xx = xx >= L ? xx - L : xx;
                site = ay * L + xx;
            }
            c.map[site] = (int32_t)(tl + i);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        ls.base = tl;
        ls.nb = B;
        reset_slots(c, ls);
        __builtin_amdgcn_wave_barrier();
        // contacts of every deposit of the batch, in deposit order:
        // c in [0,k): above (H) / left (V) of site c; [k,2k): below / right;
        // 2k: before site 0; 2k+1: after site k-1
        uint32_t ne = 0;
        int32_t cn = -1, cvx = 0, cvy = 0;
        const uint32_t total = B * nC;
        bool stop = false;
        for (uint32_t q0 = 0; q0 < total && !stop; q0 += 64) {
            uint32_t q = q0 + lane;
            bool act = q < total;
            uint32_t i = act ? fdiv(q, fC) : 0;
            uint32_t ci = q - i * nC;
            uint32_t m = tl + i;
            uint32_t am = c.banc[i];
            uint32_t om = am >> 31, site = am & 0x7FFFFFFFu;
            uint32_t ay = fdiv(site, c.fL), ax = site - ay * L;
            int32_t umx = om ? 0 : 1, umy = om ? 1 : 0;
            int32_t ii, ex, ey;
            if (ci < k) {
                ii = (int32_t)ci;
                ex = om ? -1 : 0;
                ey = om ? 0 : -1;
            } else if (ci < 2 * k) {
                ii = (int32_t)(ci - k);
                ex = om ? 1 : 0;
                ey = om ? 0 : 1;
            } else if (ci == 2 * k) {
                ii = 0;
                ex = -umx;
                ey = -umy;
            } else {
                ii = (int32_t)k - 1;
                ex = umx;
                ey = umy;
            }
            // neighbour b = anchor + ii*u_m + e (mod L)
            int32_t bx = (int32_t)ax + ii * umx + ex, by = (int32_t)ay + ii * umy + ey;
            bx = bx >= (int32_t)L ? bx - (int32_t)L : (bx < 0 ? bx + (int32_t)L : bx);
            by = by >= (int32_t)L ? by - (int32_t)L : (by < 0 ? by + (int32_t)L : by);
            int32_t n = act ? c.map[(uint32_t)by * L + (uint32_t)bx] : -1;
            bool keep = act && n >= 0 && (uint32_t)n <= m;
            int32_t vx = 0, vy = 0;
            if (keep) {
                uint32_t an = (uint32_t)n >= tl ? c.banc[(uint32_t)n - tl] : c.kmer[n];
                uint32_t on = an >> 31, ns = an & 0x7FFFFFFFu;
                uint32_t ny_ = fdiv(ns, c.fL), nx_ = ns - ny_ * L;
                int32_t j = on ? by - (int32_t)ny_ : bx - (int32_t)nx_;
                j = j < 0 ? j + (int32_t)L : j;
                int32_t unx = on ? 0 : 1, uny = on ? 1 : 0;
                // v = anchor_m - anchor_n through this contact, unwrapped
                vx = j * unx - ii * umx - ex;
                vy = j * uny - ii * umy - ey;
            }
            // drop a contact equal to the previous one on the same side
            int32_t key = keep ? n : -1;
            int32_t pn = __shfl_up(key, 1, 64), pvx = __shfl_up(vx, 1, 64), pvy = __shfl_up(vy, 1, 64);
            if (lane == 0) {
                pn = cn;
                pvx = cvx;
                pvy = cvy;
            }
            bool same_run = ci > 0 && ci < 2 * k && ci != k;
            bool emit = keep && !(same_run && pn == n && pvx == vx && pvy == vy);
            cn = __shfl(key, 63, 64);
            cvx = __shfl(vx, 63, 64);
            cvy = __shfl(vy, 63, 64);
            uint64_t bal = __ballot(emit);
            uint32_t off = (uint32_t)__popcll(bal & ((1ull << lane) - 1));
            if (emit) {
                uint32_t idx = ne + off;
                c.e_step[idx] = m;
                c.e_ms[idx] = (uint32_t)n;
                c.e_vx[idx] = vx;
                c.e_vy[idx] = vy;
            }
            ne += (uint32_t)__popcll(bal);
            __builtin_amdgcn_wave_barrier();
            if (ne + 64 > kEdges || q0 + 64 >= total) {
                process_chunk(c, ls, ne);
                ne = 0;
                if (!track && ls.nx >= 0 && ls.ny >= 0) stop = true;
                if (c.h->status != 0) stop = true;
            }
        }
        if (stop) break;
        write_back(c);
        tl = t1;
    }
    if (lane == 0) {
        c.h->nx = ls.nx;
        c.h->ny = ls.ny;
        lds_store(&c.h->lab_exit, 1u);
    }
}

// ---------------------------------------------------------------------------
// One sample, then the persistent loop
// ---------------------------------------------------------------------------

__device__ void carve(Ctx &c, const DevDesc &d, uint8_t *slab, uint8_t *lds)
{
    c.L = d.L;
    c.k = d.k;
    c.wd = d.wd;
    c.flags = d.flags;
    c.sample = d.sample;
    c.L2 = d.L * d.L;
    c.ncap = c.L2 / d.k + 1;
    c.k0 = (uint32_t)d.seed;
    c.k1 = (uint32_t)(d.seed >> 32);
    c.fL = d.fL;
    c.fk = d.fk;
    c.fC = d.fC;
    SlabLayout s = slab_layout(d.L, d.k);
    c.av[0] = (uint64_t *)(slab + s.avail0);
    c.av[1] = (uint64_t *)(slab + s.avail1);
    c.map = (int32_t *)(slab + s.map);
    c.node = (int4 *)(slab + s.node);
    c.kmer = (uint32_t *)(slab + s.kmer);
    LdsLayout l = lds_layout(d.L);
    c.h = (Hdr *)(lds + l.hdr);
    c.cnt0 = (uint32_t *)(lds + l.cnt0);
    c.cnt1 = (uint32_t *)(lds + l.cnt1);
    c.cnt2 = (uint32_t *)(lds + l.cnt2);
    c.n1 = l.n1;
    c.n2 = l.n2;
    c.ring = (uint32_t *)(lds + l.ring);
    c.banc = (uint32_t *)(lds + l.banc);
    c.e_step = (uint32_t *)(lds + l.edges);
    c.e_ms = c.e_step + kEdges;
    c.e_vx = (int32_t *)(c.e_ms + kEdges);
    c.e_vy = c.e_vx + kEdges;
    c.s_par = (uint32_t *)(lds + l.slots);
    c.s_meta = c.s_par + kSlots;
    c.s_gid = c.s_meta + kSlots;
    c.s_dx = (int32_t *)(c.s_gid + kSlots);
    c.s_dy = c.s_dx + kSlots;
    c.h_key = (uint32_t *)(lds + l.hash);
    c.h_val = c.h_key + kHash;
}

template <int NSEL>
__device__ void run_sample(const KernelArgs &a, const DevDesc &d, uint8_t *lds)
{
    constexpr uint32_t NT = 64 * (NSEL + 1);
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid >> 6;
    Ctx c;
    carve(c, d, a.slabs + (size_t)blockIdx.x * a.slab_stride, lds);
    const uint32_t L = c.L;
    const bool h_only = (c.flags & 1u) != 0;
    const bool track = (c.flags & 2u) != 0;

    // ---- initial state (Sec. II.A): all sites empty, all placements free
    {
        const size_t n2 = (size_t)c.L2;
        int4 *m4 = (int4 *)c.map;
        const size_t q4 = n2 / 4;
        for (size_t i = tid; i < q4; i += NT) m4[i] = make_int4(-1, -1, -1, -1);
        for (size_t i = q4 * 4 + tid; i < n2; i += NT) c.map[i] = -1;
        const uint32_t wd = c.wd;
        const uint32_t tailbits = L & 63u;
        const uint64_t last = tailbits ? ((1ull << tailbits) - 1) : ~0ull;
        const size_t nwords = (size_t)L * wd;
        for (size_t i = tid; i < nwords; i += NT) {
            uint32_t wi = (uint32_t)(i % wd);
            uint64_t full = wi == wd - 1 ? last : ~0ull;
            c.av[0][i] = full;
            c.av[1][i] = h_only ? 0ull : full;
        }
        const uint32_t rows = 2 * L;
        const uint32_t vcount = h_only ? 0u : L;
        for (uint32_t i = tid; i < (rows + 1) / 2; i += NT) {
            uint32_t r0 = 2 * i, r1 = 2 * i + 1;
            uint32_t c0 = r0 < L ? L : (r0 < rows ? vcount : 0);
            uint32_t c1 = r1 < L ? L : (r1 < rows ? vcount : 0);
            c.cnt0[i] = c0 | (c1 << 16);
        }
        for (uint32_t g = tid; g < c.n1; g += NT) {
            uint32_t lo = g * 64, hi = lo + 64 < rows ? lo + 64 : rows;
            uint32_t nh = hi <= L ? hi - lo : (lo >= L ? 0 : L - lo);
            c.cnt1[g] = nh * L + (hi - lo - nh) * vcount;
        }
        for (uint32_t g = tid; g < c.n2; g += NT) {
            uint32_t lo = g * 4096, hi = lo + 4096 < rows ? lo + 4096 : rows;
            uint32_t nh = hi <= L ? hi - lo : (lo >= L ? 0 : L - lo);
            c.cnt2[g] = nh * L + (hi - lo - nh) * vcount;
        }
        if (tid == 0) {
            Hdr *h = c.h;
            h->sel_progress = 0;
            h->sel_done = 0;
            h->lab_progress = 0;
            h->lab_exit = 0;
            h->clr_gen = 0;
            h->clr_done = 0;
            h->cur_p = 0;
            h->nslots = 0;
            h->nx = -1;
            h->ny = -1;
            h->nclusters = 0;
            h->nonwrap = 0;
            h->status = 0;
            h->wchg = 0;
            h->occ = 0;
            h->seqh = 0;
        }
    }
    __syncthreads();

    // ---- the two chains
    if (wave == 0)
        selector<NSEL>(c);
    else if (wave < (uint32_t)NSEL)
        helper<NSEL>(c, wave);
    else
        labeler(c, track);
    __syncthreads();

    // ---- cluster census at jamming (Appendix A)
    const uint32_t njam = c.h->sel_done - 1;
    if (track) {
        uint32_t roots = 0, nonwrap = 0;
        for (uint32_t i = tid; i < njam; i += NT) {
            int4 nd = c.node[i];
            if ((uint32_t)nd.x == i) {
                ++roots;
                if ((nd.w & 0x300) == 0) ++nonwrap;
            }
        }
        atomicAdd(&c.h->nclusters, roots);
        atomicAdd(&c.h->nonwrap, nonwrap);
        __syncthreads();
    }
    if (tid == 0) {
        DevResult r;
        const uint64_t Lw = L, kw = c.k;
        r.n_jam = njam;
        r.n_wrap_x = c.h->nx;
        r.n_wrap_y = c.h->ny;
        int64_t any = -1;
        if (r.n_wrap_x > 0) any = r.n_wrap_x;
        if (r.n_wrap_y > 0 && (any < 0 || r.n_wrap_y < any)) any = r.n_wrap_y;
        r.n_wrap_any = any;
        r.occ_hash = c.h->occ;
        r.seq_hash = c.h->seqh;
        r.n_clusters_jam = track ? (int32_t)c.h->nclusters : -1;
        r.n_nonwrapping_jam = track ? (int32_t)c.h->nonwrap : -1;
        r.status = c.h->status;
        r.tile = (int32_t)a.tile;
        r.wchg_words = c.h->wchg;
        r.alg_bytes = 4 * Lw * Lw + 16 * Lw * c.wd +
                      (uint64_t)njam * (4 * kw + 4 * (2 * kw + 2) + 8 * c.wd + 16) + 16 * r.wchg_words;
        a.results[d.out] = r;
    }
    __syncthreads();
}

template <int NSEL>
__global__ __launch_bounds__(64 * (NSEL + 1)) void rsa_persistent(KernelArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t i = next;
        __syncthreads();
        if (i >= a.n) return;
        const DevDesc d = a.descs[i];
        run_sample<NSEL>(a, d, lds);
    }
}

__global__ void rsa_reset_queues(uint32_t *queues, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) queues[i] = 0;
}

}  // namespace rsa

// Host-visible launch table.
namespace rsa {
using KernelFn = void (*)(KernelArgs);
extern const void *kPersistentKernels[kNumTiles];
const void *kPersistentKernels[kNumTiles] = {
    (const void *)&rsa_persistent<kTileWaves[0]>, (const void *)&rsa_persistent<kTileWaves[1]>,
    (const void *)&rsa_persistent<kTileWaves[2]>, (const void *)&rsa_persistent<kTileWaves[3]>,
    (const void *)&rsa_persistent<kTileWaves[4]>};
const void *kResetKernel = (const void *)&rsa_reset_queues;
}  // namespace rsa
