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

#ifndef RSA_TU_WAVES
#error "define RSA_TU_WAVES: the wave-count index (0 .. kNumWaveTiles - 1) this unit instantiates"
#endif

namespace rsa {

// Internal failure codes reported in the result's status field.  They mean a
// broken invariant (counts that disagree with the bitmaps, a cycle in the
// union-find); the sample then stops instead of reading out of bounds.
constexpr int32_t kErrSelect = -100;
constexpr int32_t kErrLabel = -101;
constexpr uint32_t kMaxHops = 64;   // union by rank keeps trees below log2(L^2) levels
constexpr uint32_t kSideGather = 512;   // k from which contacts are gathered side by side
                                        // (sparse-clear kernels)

// Loads whose latency must overlap other work are typed as global memory.
// The slab pointers reach the kernel inside a struct, so the compiler cannot
// infer their address space and emits FLAT loads; a FLAT result is waited
// for with vmcnt(0), i.e. together with every load issued after it.
template <class T>
using gmem = __attribute__((address_space(1))) T;

__device__ __forceinline__ uint32_t gld32(const uint32_t *p) { return *(const gmem<uint32_t> *)p; }
__device__ __forceinline__ void gst32(uint32_t *p, uint32_t v) { *(gmem<uint32_t> *)p = v; }
__device__ __forceinline__ void gst64(uint64_t *p, uint64_t v) { *(gmem<uint64_t> *)p = v; }
__device__ __forceinline__ void gand64(uint64_t *p, uint64_t m)
{
    __hip_atomic_fetch_and((gmem<unsigned long long> *)p, (unsigned long long)m, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// v[i] of four values (i wave-uniform or a constant), without an array
// indexed at run time (which would live in scratch memory).
template <class T>
__device__ __forceinline__ T pick4(uint32_t i, T a, T b, T c, T d)
{
    return i == 0 ? a : i == 1 ? b : i == 2 ? c : d;
}

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

// Inclusive prefix sum over the 64 lanes with DPP moves: shifts by 1, 2, 4, 8
// inside each 16-lane row, then broadcasts of lane 15 and lane 31 into the
// rows above (four times cheaper than LDS-crossbar shuffles).
__device__ __forceinline__ uint32_t wave_scan(uint32_t v)
{
    v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return v;
}

// Value of a wave-uniform lane (scalar read, no LDS traffic).
// (readlane returns int: go through uint32_t so that nothing sign-extends)
__device__ __forceinline__ uint32_t bcast(uint32_t v, uint32_t lane)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)lane);
}

__device__ __forceinline__ uint64_t bcast64(uint64_t v, uint32_t lane)
{
    const uint32_t lo = bcast((uint32_t)v, lane), hi = bcast((uint32_t)(v >> 32), lane);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) { return bcast(wave_scan(v), 63); }

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v)
{
#pragma unroll
    for (uint32_t d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t first_lane(uint64_t ballot) { return (uint32_t)(__ffsll((long long)ballot) - 1); }

// Set bits of `ballot` below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t ballot)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
}

// The previous lane's v (DPP wave shift right by one); lane 0 gets `first`.
__device__ __forceinline__ int32_t from_previous_lane(int32_t v, int32_t first)
{
    return __builtin_amdgcn_update_dpp(first, v, 0x138, 0xf, 0xf, false);
}

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
    uint32_t t0;             // first step of this run (0, or where it resumed)
    uint32_t p0;             // placement of step t0 on resume; on yield, of
                             // the step the run stopped before
    unsigned long long wchg;
    unsigned long long occ;
    unsigned long long seqh;
    uint32_t resumed;        // state restored from the slab
    uint32_t preempt;        // the selecting wave stopped at its deadline
    uint32_t lab_stop;       // labelling ended early (both wrap steps known)
    uint32_t stop;           // selection ends before this step (0 = at jamming)
    unsigned long long ncon[3];   // contact census: both H, both V, perpendicular
    unsigned long long sel_acc[10];  // selecting wave's phase counters (profiling)
    uint32_t bar;            // interval clear: arrivals of the selecting waves at the mid-step barrier
    uint32_t jrs, jn;        // interval clear: V anchors a vertical deposit removed from its own column
};

// Selecting-wave profile accumulators, kept in LDS rather than in registers.
enum SelAcc { kAccStart = 0, kAccRing, kAccSelect, kAccClear, kAccHook, kAccProcess, kAccSpec, kAccIvCut, kAccIvMeet,
              kAccIvRows };

struct Ctx {
    unsigned long long *prof;   // this sample's counters, or null
    uint32_t L, k, wd, flags, sample;
    uint32_t ncap;     // k-mer records in the slab, L*L/k + 1
    uint32_t k0, k1;   // Philox key
    // bitmap tiles: 2^lg_tr rows x 2^(4-lg_tr) words; site-map tiles:
    // 2^lg_mr rows x 2^(5-lg_mr) sites (the rest is derived on use, which
    // keeps the scalar registers of the selecting wave free)
    uint32_t lg_tr, lg_mr;
    uint32_t spec_rows;
    FastDiv fL, fk, fC, fwd, fwp;
    uint64_t *av0, *av1;   // availability bitmaps of H / V placements
    uint64_t *sm0, *sm1;   // their summary bits (sparse clear only)
    int32_t *map;
    int4 *node;
    uint32_t *kmer;
    Hdr *h;
    uint32_t *cnt0, *cnt1, *cnt2;
    uint32_t *ring, *banc;
    uint32_t *e_step;   // edge lists: step, then ms, vx, vy (kEdges each)
    uint32_t *s_par;    // local union-find: parent, then meta, gid, dx, dy (kSlots each)
    uint32_t *h_key;    // root hash: keys, then values (kHash each)
    // interval clear (long k-mers): anchor-interval buckets of H rows and V
    // columns in the slab, per-row difference counts of a block and their
    // 64-row sums in LDS, or (ivg) two sets of them in the slab, set t & 1
    // at dD + (t & 1) * ivstride for step t
    uint32_t interval, ivg, ivstride;
    uint32_t *hb, *vb;
    uint32_t *dD, *dC;
    FastDiv fB;
    // compressed lattice (long k-mers): occupancy and anchor bitmaps and the
    // placement -> deposit table instead of the site map
    uint32_t compressed, nlw, nt16, hlg;
    uint64_t *ohr, *ovr, *ohc, *ovc, *ahr, *avc;
    unsigned long long *khash;

    __device__ __forceinline__ uint32_t L2() const { return L * L; }
    __device__ __forceinline__ uint32_t wp() const { return padded_words(L); }
    __device__ __forceinline__ uint32_t lp() const { return padded_side(L); }
    __device__ __forceinline__ uint32_t swp() const { return summary_words(L); }
    __device__ __forceinline__ uint32_t n1() const { return (2 * L + 63) / 64; }
    __device__ __forceinline__ uint32_t n2() const { return (2 * L + 4095) / 4096; }
    __device__ __forceinline__ uint32_t lg_tw() const { return 4 - lg_tr; }
    __device__ __forceinline__ uint32_t tr_m() const { return (1u << lg_tr) - 1; }
    __device__ __forceinline__ uint32_t tw_m() const { return (1u << (4 - lg_tr)) - 1; }
    __device__ __forceinline__ uint32_t tpr() const { return padded_words(L) >> (4 - lg_tr); }
    __device__ __forceinline__ uint32_t lg_mc() const { return 5 - lg_mr; }
    __device__ __forceinline__ uint32_t mr_m() const { return (1u << lg_mr) - 1; }
    __device__ __forceinline__ uint32_t mc_m() const { return (1u << (5 - lg_mr)) - 1; }
    __device__ __forceinline__ uint32_t mtpr() const { return padded_side(L) >> (5 - lg_mr); }
    __device__ __forceinline__ uint32_t *e_ms() const { return e_step + kEdges; }
    __device__ __forceinline__ int32_t *e_vx() const { return (int32_t *)(e_step + 2 * kEdges); }
    __device__ __forceinline__ int32_t *e_vy() const { return (int32_t *)(e_step + 3 * kEdges); }
    __device__ __forceinline__ uint32_t *s_meta() const { return s_par + kSlots; }
    __device__ __forceinline__ uint32_t *s_gid() const { return s_par + 2 * kSlots; }
    __device__ __forceinline__ int32_t *s_dx() const { return (int32_t *)(s_par + 3 * kSlots); }
    __device__ __forceinline__ int32_t *s_dy() const { return (int32_t *)(s_par + 4 * kSlots); }
    __device__ __forceinline__ uint32_t *h_val() const { return h_key + kHash; }
};

__device__ __forceinline__ uint64_t *bitmap(const Ctx &c, uint32_t o) { return o ? c.av1 : c.av0; }

// Word w of bitmap row `row` inside its 128-byte tile.
// (32-bit: a bitmap holds at most 32768 x 528 words, a map 2^30 sites)
__device__ __forceinline__ uint32_t bm_index(const Ctx &c, uint32_t row, uint32_t w)
{
    return (((row >> c.lg_tr) * c.tpr() + (w >> c.lg_tw())) << 4) + ((row & c.tr_m()) << c.lg_tw()) +
           (w & c.tw_m());
}

// Site (y, x) of the map inside its 128-byte tile.
__device__ __forceinline__ uint32_t map_index(const Ctx &c, uint32_t y, uint32_t x)
{
    return (((y >> c.lg_mr) * c.mtpr() + (x >> c.lg_mc())) << 5) + ((y & c.mr_m()) << c.lg_mc()) +
           (x & c.mc_m());
}

__device__ __forceinline__ uint64_t tick() { return (uint64_t)wall_clock64(); }

__device__ __forceinline__ void prof_add(const Ctx &c, int slot, uint64_t v)
{
    if (c.prof && lane_id() == 0) atomicAdd(&c.prof[slot], (unsigned long long)v);
}

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

// A rectangle of placements to make unavailable: orientation o, anchor rows
// row0 .. row0+nrows-1 (mod L) and anchor columns in the cyclic interval
// [c0, c0+len).  Its items are (row, word) pairs: the columns touch words
// a0 .. a0+nA-1 and, past the seam, words 0 .. nw-nA-1, each word once.
struct Rect {
    uint32_t o, row0, nrows, c0, len;
    uint32_t a0, nA, nw;
    uint32_t lg;      // nw <= 64: 1 << lg lanes per row; else all ones
};

__device__ __forceinline__ Rect make_rect(const Ctx &c, uint32_t o, uint32_t row0, uint32_t nrows,
                                          uint32_t c0, uint32_t len)
{
    const uint32_t L = c.L;
    Rect r;
    r.o = o;
    r.row0 = row0;
    r.nrows = nrows;
    r.c0 = c0;
    r.len = len;
    if (len >= L) {
        r.a0 = 0;
        r.nA = c.wd;
        r.nw = c.wd;
    } else {
        uint32_t end = c0 + len;
        uint32_t endA = end < L ? end : L;
        r.a0 = c0 >> 6;
        r.nA = ((endA - 1) >> 6) - r.a0 + 1;
        uint32_t nB = 0;
        if (end > L) {
            uint32_t b1 = (end - L - 1) >> 6;
            nB = (b1 == r.a0) ? b1 : b1 + 1;
        }
        r.nw = r.nA + nB;
    }
    r.lg = r.nw <= 64 ? (r.nw <= 1 ? 0 : 32 - __clz(r.nw - 1)) : 0xFFFFFFFFu;
    return r;
}

// Deposit of k-mer (o, y, x): every placement covering one of its sites stops
// being available (Sec. II.B).  Horizontal at (y, x): H anchors in row y,
// columns x-k+1 .. x+k-1, and V anchors in rows y-k+1 .. y, columns
// x .. x+k-1.  Vertical: the transpose.  Runs longer than L wrap once.
struct Clear {
    Rect a, b;
};

__device__ __forceinline__ Clear make_clear(const Ctx &c, uint32_t o, uint32_t y, uint32_t x)
{
    const uint32_t L = c.L, k = c.k;
    uint32_t strip = 2 * k - 1 < L ? 2 * k - 1 : L;
    uint32_t back = x + L - (k - 1);
    back = back >= L ? back - L : back;
    uint32_t up = y + L - (k - 1);
    up = up >= L ? up - L : up;
    Clear cl;
    if (o == 0) {
        cl.a = make_rect(c, 0, y, 1, back, strip);
        cl.b = make_rect(c, 1, up, k, x, k);
    } else {
        cl.a = make_rect(c, 1, up, strip, x, 1);
        cl.b = make_rect(c, 0, y, k, back, k);
    }
    return cl;
}

// One lane's fixed part of a rectangle.  Narrow rectangles (nw <= 64) give
// every lane one word column: lanes are grouped 2^lg per row, so the lane's
// word, mask and tile-column offset are the same in every row it visits.
// Wide rectangles visit one row per round, 64 words at a time.
struct RectLane {
    uint32_t rounds;     // wave-uniform number of rounds for this wave
    uint32_t rsub, rows_per;
    uint32_t w, colpart;
    uint64_t mask;
    uint32_t nchunk;     // wide: 64-word chunks per row
};

// NARROW: every row has at most 64 words (L <= 4096), so no rectangle is
// wide and the wide path is compiled out.
template <bool NARROW>
__device__ __forceinline__ RectLane rect_lane(const Ctx &c, const Rect &r, uint32_t wv, uint32_t nwv)
{
    const uint32_t lane = lane_id();
    RectLane rl;
    if (NARROW || r.lg != 0xFFFFFFFFu) {
        rl.rows_per = 64u >> r.lg;
        rl.rsub = lane >> r.lg;
        const uint32_t wsub = lane & ((1u << r.lg) - 1);
        rl.w = wsub < r.nA ? r.a0 + wsub : wsub - r.nA;
        rl.mask = wsub < r.nw ? col_mask(c.L, r.c0, r.len, rl.w) : 0;
        rl.colpart = ((rl.w >> c.lg_tw()) << 4) + (rl.w & c.tw_m());
        const uint32_t all = (r.nrows + rl.rows_per - 1) / rl.rows_per;   // row groups
        rl.rounds = all > wv ? (all - wv + nwv - 1) / nwv : 0;
        rl.nchunk = 0;
    } else {
        rl.nchunk = (r.nw + 63) >> 6;
        const uint32_t all = r.nrows * rl.nchunk;
        rl.rounds = all > wv ? (all - wv + nwv - 1) / nwv : 0;
        rl.rsub = rl.rows_per = rl.w = rl.colpart = 0;
        rl.mask = 0;
    }
    return rl;
}

// Round rr of wave wv: the word this lane reads (row, bitmap index, mask).
template <bool NARROW>
__device__ __forceinline__ bool rect_round(const Ctx &c, const Rect &r, const RectLane &rl, uint32_t rr,
                                           uint32_t wv, uint32_t nwv, uint32_t &row, uint32_t &at,
                                           uint64_t &mask)
{
    const uint32_t g = rr * nwv + wv;   // wave-uniform
    uint32_t i, w;
    if (NARROW || rl.nchunk == 0) {
        i = g * rl.rows_per + rl.rsub;
        mask = rl.mask;
        w = rl.w;
        if (i >= r.nrows || mask == 0) return false;
        row = r.row0 + i;
        row = row >= c.L ? row - c.L : row;
        at = (((row >> c.lg_tr) * c.tpr()) << 4) + ((row & c.tr_m()) << c.lg_tw()) + rl.colpart;
        return true;
    }
    i = g / rl.nchunk;
    const uint32_t j = (g - i * rl.nchunk) * 64 + lane_id();
    if (j >= r.nw) return false;
    w = j < r.nA ? r.a0 + j : j - r.nA;
    mask = col_mask(c.L, r.c0, r.len, w);
    row = r.row0 + i;
    row = row >= c.L ? row - c.L : row;
    at = bm_index(c, row, w);
    return true;
}

struct NoHook {
    __device__ __forceinline__ void operator()() const {}
};

// Wave wv of nwv clears its share of both rectangles, CAP words in flight
// per lane: read the words, clear the blocked bits that are still set,
// decrement the row counts by the bits cleared.  hook() runs while the first
// CAP reads are in flight; it may read LDS but not global memory (its
// instructions then overlap the reads' latency).  landed() runs once those
// reads are in, before their writes: loads it issues stay in flight through
// the writes (no later wait covers them).
template <int CAP, bool NARROW, typename Hook = NoHook, typename Hook2 = NoHook>
__device__ __forceinline__ void clear_items(const Ctx &c, const Clear &cl, uint32_t wv, uint32_t nwv,
                                            uint32_t &wchg, const Hook &hook = Hook(),
                                            const Hook2 &landed = Hook2())
{
    const RectLane la = rect_lane<NARROW>(c, cl.a, wv, nwv);
    const RectLane lb = rect_lane<NARROW>(c, cl.b, wv, nwv);
    const uint32_t total = la.rounds + lb.rounds;
    uint64_t *const bma = bitmap(c, cl.a.o);
    uint64_t *const bmb = bitmap(c, cl.b.o);
    const uint32_t rba = cl.a.o * c.L, rbb = cl.b.o * c.L;
    if (total == 0) {
        hook();
        landed();
        return;
    }
    // the first batch is peeled off the loop, so that its hooks sit in
    // straight-line code between its reads and its writes
    const auto batch = [&](uint32_t base, auto first) {
        // each lane's CAP words: address, mask of the blocked bits and count
        // row are kept from the reads to the writes
        uint64_t old[CAP], msk[CAP];
        uint32_t idx[CAP], crow[CAP];
#pragma unroll
        for (int s = 0; s < CAP; ++s) {
            const uint32_t rr = base + s;
            uint32_t row = 0;
            uint32_t at = 0;
            uint64_t mask = 0;
            bool ok = false;
            const bool in_a = rr < la.rounds;
            if (in_a)
                ok = rect_round<NARROW>(c, cl.a, la, rr, wv, nwv, row, at, mask);
            else if (rr < total)
                ok = rect_round<NARROW>(c, cl.b, lb, rr - la.rounds, wv, nwv, row, at, mask);
            old[s] = ok ? ((const gmem<uint64_t> *)(in_a ? bma : bmb))[at] : 0;
            msk[s] = ok ? mask : 0;
            idx[s] = (uint32_t)at;
            crow[s] = (in_a ? rba : rbb) + row;
        }
        if constexpr (decltype(first)::value) {
            hook();
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this batch's reads have landed
            landed();
        }
#pragma unroll
        for (int s = 0; s < CAP; ++s) {
            const uint64_t hit = old[s] & msk[s];
            if (hit) {
                (base + s < la.rounds ? bma : bmb)[idx[s]] = old[s] & ~hit;
                count_sub(c, crow[s], (uint32_t)__popcll(hit));
                ++wchg;
            }
        }
    };
    batch(0u, std::true_type());
    for (uint32_t base = CAP; base < total; base += CAP) batch(base, std::false_type());
}

// Sparse clear of one rectangle.  Per row, the rectangle's words fall in one
// or a few summary words (64 words each); an item is one (row, summary word).
// A wave's lanes take CAP items at once: read their summary words, keep the
// bits of the rectangle's words that may still be non-zero, then read only
// those data words (up to DCAP in flight per lane per round), clear the
// blocked bits, and drop the summary bit of every word that became zero.
__device__ __forceinline__ uint32_t rect_summary_words(const Rect &r, uint32_t &nsA)
{
    nsA = ((r.a0 + r.nA - 1) >> 6) - (r.a0 >> 6) + 1;
    const uint32_t nB = r.nw - r.nA;
    return nsA + (nB ? ((nB - 1) >> 6) + 1 : 0);
}

template <int CAP, int DCAP>
__device__ __forceinline__ void sparse_rect(const Ctx &c, const Rect &r, uint32_t wv, uint32_t nwv,
                                            uint32_t &wchg)
{
    const uint32_t lane = lane_id(), L = c.L;
    uint32_t nsA;
    const uint32_t ns = rect_summary_words(r, nsA);
    const uint32_t nB = r.nw - r.nA;
    const uint32_t items = r.nrows * ns;
    uint64_t *const bm = bitmap(c, r.o);
    uint64_t *const sm = r.o ? c.sm1 : c.sm0;
    const uint32_t rowbase = r.o * L;
    for (uint32_t base = wv * 64; base < items; base += nwv * 64 * CAP) {
        uint64_t cand[CAP], zero[CAP];
        uint32_t srow[CAP], ssw[CAP];
#pragma unroll
        for (int s = 0; s < CAP; ++s) {
            const uint32_t f = base + (uint32_t)s * nwv * 64 + lane;
            uint64_t bits = 0;
            uint32_t row = 0, sw = 0;
            if (f < items) {
                const uint32_t i = f / ns, j = f - i * ns;
                row = r.row0 + i;
                row = row >= L ? row - L : row;
                uint32_t lo, hi;   // data words of this item, [lo, hi)
                if (j < nsA) {
                    sw = (r.a0 >> 6) + j;
                    lo = sw * 64 > r.a0 ? sw * 64 : r.a0;
                    hi = sw * 64 + 64 < r.a0 + r.nA ? sw * 64 + 64 : r.a0 + r.nA;
                } else {
                    sw = j - nsA;
                    lo = sw * 64;
                    hi = sw * 64 + 64 < nB ? sw * 64 + 64 : nB;
                }
                const uint32_t b0 = lo - sw * 64, b1 = hi - sw * 64;
                bits = (b1 == 64 ? ~0ull : ((1ull << b1) - 1)) & ~((1ull << b0) - 1);
            }
            srow[s] = row;
            ssw[s] = sw;
            cand[s] = bits;
            zero[s] = 0;
        }
#pragma unroll
        for (int s = 0; s < CAP; ++s)
            if (cand[s]) cand[s] &= sm[srow[s] * c.swp() + ssw[s]];
        // data words, DCAP per lane per round
        for (;;) {
            bool any = false;
#pragma unroll
            for (int s = 0; s < CAP; ++s) any = any || cand[s] != 0;
            if (__ballot(any) == 0) break;
            uint64_t old[DCAP];
            uint32_t pick[DCAP];   // item << 8 | word bit, or ~0
            uint32_t dat[DCAP], dw[DCAP], drow[DCAP];   // word index, word column, row
#pragma unroll
            for (int d = 0; d < DCAP; ++d) {
                pick[d] = 0xFFFFFFFFu;
                old[d] = 0;
                dat[d] = dw[d] = drow[d] = 0;
#pragma unroll
                for (int s = 0; s < CAP; ++s) {
                    if (pick[d] == 0xFFFFFFFFu && cand[s] != 0) {
                        const uint32_t b = (uint32_t)(__ffsll((long long)cand[s]) - 1);
                        cand[s] &= cand[s] - 1;
                        pick[d] = ((uint32_t)s << 8) | b;
                        dw[d] = ssw[s] * 64 + b;
                        drow[d] = srow[s];
                        dat[d] = bm_index(c, srow[s], dw[d]);
                        old[d] = bm[dat[d]];
                    }
                }
            }
#pragma unroll
            for (int d = 0; d < DCAP; ++d) {
                if (pick[d] == 0xFFFFFFFFu) continue;
                const uint32_t s = pick[d] >> 8, b = pick[d] & 255u;
                const uint32_t row = drow[d], w = dw[d];
                const uint64_t hit = old[d] & col_mask(L, r.c0, r.len, w);
                if (hit) {
                    const uint64_t nv = old[d] & ~hit;
                    bm[dat[d]] = nv;
                    count_sub(c, rowbase + row, (uint32_t)__popcll(hit));
                    ++wchg;
                    if (nv == 0) {
#pragma unroll
                        for (int q = 0; q < CAP; ++q)
                            if ((uint32_t)q == s) zero[q] |= 1ull << b;
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < CAP; ++s)
            if (zero[s]) atomicAnd((unsigned long long *)&sm[srow[s] * c.swp() + ssw[s]], ~zero[s]);
    }
}

template <int CAP>
__device__ __forceinline__ void sparse_clear(const Ctx &c, const Clear &cl, uint32_t wv, uint32_t nwv,
                                             uint32_t &wchg)
{
    (void)CAP;   // four summary words and eight data words in flight per lane
    sparse_rect<4, 8>(c, cl.a, wv, nwv, wchg);
    sparse_rect<4, 8>(c, cl.b, wv, nwv, wchg);
}

// ---------------------------------------------------------------------------
// Interval clear (long k-mers)
// ---------------------------------------------------------------------------
// A deposit makes unavailable every placement covering one of its sites
// (Sec. II.B).  On one line (a row of H anchors or a column of V anchors)
// those are the available anchors inside one cyclic range: the deposit's own
// line loses [x-k+1, x+k-1] (its strip), each of the k lines it crosses loses
// [x-k+1, x] (its row or column of the block).  A line's available anchors
// live in buckets of k+1 positions, one interval piece each at most, so a
// line's cut reads the two to four bucket entries its range touches and
// writes back those that change: the k+1 lines of a deposit are cut side by
// side in one round trip, with exact counts and without reading a bitmap.
// V anchors are also kept in the row-major bitmap the select reads (within a
// V row the canonical order runs across the columns); H rows are selected
// from their buckets.

// Result of cutting one line.
struct LineCut {
    uint32_t n;       // anchors removed
    uint32_t nw;      // 64-bit words of the line's canonical bitmap row holding them
    uint32_t start;   // first removed anchor in cyclic order (when n > 0)
    bool bad;         // a bucket would keep two pieces: broken invariant
};

__device__ __forceinline__ uint32_t seg_start(uint32_t v) { return v & 0xFFFFu; }
__device__ __forceinline__ uint32_t seg_end(uint32_t v) { return v >> 16; }

// The buckets a cut of the cyclic range [lo, lo + len) (len >= L: the whole
// line) touches, in increasing order: buckets 0 .. n0 - 1 (the part past the
// seam), then ja, ja + 1, ...; nj in all, at most four, as the range is
// shorter than two buckets and the seam splits it at most once.  The same for
// every line cut with that range.  (Plain fields only: an array indexed at
// run time would live in scratch memory.)
struct CutPlan {
    uint32_t lo, len, wend;
    uint32_t n0, ja, nj;
    uint32_t off0, off1, off2, off3;   // list offsets of the touched buckets' entries of line 0
    bool full, wraps, over;
};

__device__ __forceinline__ uint32_t plan_bucket(const CutPlan &p, uint32_t i)
{
    return i < p.n0 ? i : p.ja + (i - p.n0);
}

__device__ __forceinline__ CutPlan cut_plan(const Ctx &c, uint32_t lo, uint32_t len)
{
    const uint32_t L = c.L;
    CutPlan p;
    p.lo = lo;
    p.len = len;
    p.full = len >= L;
    p.wraps = !p.full && lo + len > L;
    p.wend = p.wraps ? lo + len - L : 0;   // the range's part past the seam: [0, wend)
    uint32_t jb;
    p.n0 = 0;
    if (p.full) {
        p.ja = 0;
        jb = fdiv(L - 1, c.fB);
    } else if (p.wraps) {
        const uint32_t jw = fdiv(p.wend - 1, c.fB);
        p.n0 = jw + 1;
        const uint32_t j0 = fdiv(lo, c.fB);
        p.ja = j0 > jw + 1 ? j0 : jw + 1;
        jb = fdiv(L - 1, c.fB);
    } else {
        p.ja = fdiv(lo, c.fB);
        jb = fdiv(lo + len - 1, c.fB);
    }
    const uint32_t n1 = jb >= p.ja ? jb - p.ja + 1 : 0;
    p.nj = p.n0 + n1;
    p.over = p.nj > 4;
    if (p.over) p.nj = 4;
    const uint32_t lp = c.lp();
    p.off0 = plan_bucket(p, 0) * lp;
    p.off1 = plan_bucket(p, 1) * lp;
    p.off2 = plan_bucket(p, 2) * lp;
    p.off3 = plan_bucket(p, 3) * lp;
    return p;
}

// Read the touched bucket entries of line q (kNoSeg where nothing is read).
// Every lane loads (an inactive one from line 0, discarded), so the loads
// need no per-lane branches; entries past the plan are skipped for the wave.
__device__ __forceinline__ void cut_load(const Ctx &c, const CutPlan &p, const uint32_t *list, uint32_t q, bool act,
                                         uint32_t ev[4])
{
    const uint32_t *const base = list + (act ? q : 0u);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t v = kNoSeg;
        if ((uint32_t)i < p.nj) v = gld32(base + pick4((uint32_t)i, p.off0, p.off1, p.off2, p.off3));
        ev[i] = act ? v : kNoSeg;
    }
}

// Remove the available anchors inside the plan's range from line q, whose
// touched entries are ev: every touched bucket keeps what lies outside the
// range, and the entries that change are written back.
__device__ __forceinline__ LineCut cut_apply(const Ctx &c, const CutPlan &p, uint32_t *list, uint32_t q, bool act,
                                             const uint32_t ev[4])
{
    const uint32_t lo = p.lo, len = p.len, wend = p.wend;
    LineCut r;
    r.n = 0;
    r.nw = 0;
    r.start = 0;
    r.bad = act && p.over;
    int32_t lastw = -1;
    uint32_t prev_e = 0;
    bool first = true;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t E = ev[i];
        if (E == kNoSeg) continue;
        const int32_t s = (int32_t)seg_start(E), e = (int32_t)seg_end(E);
        // the part of the piece outside the range stays (one interval at most)
        int32_t ks = 1, ke = 0;
        if (!p.full) {
            if (p.wraps) {   // outside: [wend, lo)
                const int32_t a = s > (int32_t)wend ? s : (int32_t)wend;
                const int32_t b = e < (int32_t)lo - 1 ? e : (int32_t)lo - 1;
                if (a <= b) {
                    ks = a;
                    ke = b;
                }
            } else {         // outside: [lo + len, L) and [0, lo)
                const int32_t ca = (int32_t)(lo + len);
                const int32_t a1 = s > ca ? s : ca;
                const int32_t b2 = e < (int32_t)lo - 1 ? e : (int32_t)lo - 1;
                const bool k1 = a1 <= e;
                const bool k2 = s <= b2;
                if (k1 && k2) r.bad = true;
                if (k1) {
                    ks = a1;
                    ke = e;
                } else if (k2) {
                    ks = s;
                    ke = b2;
                }
            }
        }
        const bool keep = ks <= ke;
        // removed pieces, in increasing position
        int32_t ps0 = s, pe0 = e, ps1 = 0, pe1 = -1;
        if (keep) {
            pe0 = ks - 1;   // left of what stays (empty if ks == s)
            ps1 = ke + 1;   // right of it (empty if ke == e)
            pe1 = e;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int32_t a = h ? ps1 : ps0, b = h ? pe1 : pe0;
            if (a > b) continue;
            r.n += (uint32_t)(b - a + 1);
            int32_t w0 = a >> 6;
            const int32_t w1 = b >> 6;
            if (w0 <= lastw) w0 = lastw + 1;
            if (w1 >= w0) r.nw += (uint32_t)(w1 - w0 + 1);
            if (w1 > lastw) lastw = w1;
            // the cyclic start follows the gap between two removed pieces,
            // if there is one; otherwise it is the first piece
            if (first || (uint32_t)a != prev_e + 1) r.start = (uint32_t)a;
            first = false;
            prev_e = (uint32_t)b;
        }
        const uint32_t nv = keep ? ((uint32_t)ks | ((uint32_t)ke << 16)) : kNoSeg;
        if (nv != E) gst32(&list[pick4((uint32_t)i, p.off0, p.off1, p.off2, p.off3) + q], nv);
    }
    return r;
}

// Wave-wide minimum / maximum / OR.
__device__ __forceinline__ uint32_t wave_min32(uint32_t v)
{
#pragma unroll
    for (uint32_t d = 32; d >= 1; d >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, (int)d, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_max32(uint32_t v)
{
#pragma unroll
    for (uint32_t d = 32; d >= 1; d >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, (int)d, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_or32(uint32_t v)
{
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v |= __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return bcast(v, 63);
}

// Bits a..b (0 <= a, b <= 63) of a word, or 0 when a > b.
__device__ __forceinline__ uint64_t bit_range(int32_t a, int32_t b)
{
    if (a > b) return 0;
    return (~0ull >> (63 - b)) & (~0ull << a);
}

// Subtract v from the count of canonical row R for every lane with `act`:
// the row counts lane by lane, their 64-row and 4096-row sums once per
// distinct 64-row group of the wave.
__device__ __forceinline__ void count_sub_wave(const Ctx &c, bool act, uint32_t R, uint32_t v)
{
    const bool on = act && v != 0;
    if (on) atomicSub(&c.cnt0[R >> 1], v << ((R & 1) << 4));
    uint64_t pend = __ballot(on);
    while (pend) {
        const uint32_t g = bcast(R >> 6, first_lane(pend));
        const bool in = on && (R >> 6) == g;
        const uint32_t sum = wave_sum32(in ? v : 0u);
        if (lane_id() == 0) {
            atomicSub(&c.cnt1[g], sum);
            atomicSub(&c.cnt2[g >> 6], sum);
        }
        pend &= ~__ballot(in);
    }
}

// The selecting waves meet once per step between the two phases of the
// interval clear (LDS arrivals counter; every wave passes the same number).
template <int NSEL>
__device__ __forceinline__ void sel_barrier(const Ctx &c, uint32_t &passed, bool selecting)
{
    if constexpr (NSEL > 1) {
        ++passed;
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (lane_id() == 0) atomicAdd(&c.h->bar, 1u);
        // a wave that waits yields its SIMD's issue slots to the waves still working
        __builtin_amdgcn_s_setprio(0);
        while (lds_load(&c.h->bar) < passed * (uint32_t)NSEL) __builtin_amdgcn_s_sleep(1);
        if (selecting)
            __builtin_amdgcn_s_setprio(3);
        else
            __builtin_amdgcn_s_setprio(2);
    }
}

// Aligned 64-blocks of line indices covering the cyclic span [q0, q0 + k):
// the part past the seam [0, q0 + k - L) first, then [q0, ...); a block both
// parts touch is listed once.
struct Span {
    uint32_t q0, k;
    uint32_t e2;       // blocks 0 .. e2 - 1 come from the part past the seam
    uint32_t s1, n;    // then blocks s1, s1 + 1, ...; n blocks in all
};

__device__ __forceinline__ Span make_span(const Ctx &c, uint32_t q0, uint32_t k)
{
    const uint32_t L = c.L;
    Span sp;
    sp.q0 = q0;
    sp.k = k;
    const uint32_t end1 = q0 + k < L ? q0 + k : L;
    const uint32_t b1 = q0 >> 6, l1 = (end1 - 1) >> 6;
    if (q0 + k > L) {
        const uint32_t l2 = (q0 + k - L - 1) >> 6;
        sp.e2 = l2 + 1;
        sp.s1 = b1 > l2 ? b1 : l2 + 1;
        sp.n = sp.e2 + (l1 >= sp.s1 ? l1 - sp.s1 + 1 : 0);
    } else {
        sp.e2 = 0;
        sp.s1 = b1;
        sp.n = l1 - b1 + 1;
    }
    return sp;
}

__device__ __forceinline__ uint32_t span_block(const Span &sp, uint32_t m)
{
    return m < sp.e2 ? m : sp.s1 + (m - sp.e2);
}

__device__ __forceinline__ bool in_span(const Ctx &c, const Span &sp, uint32_t q)
{
    if (q >= c.L) return false;
    uint32_t d = q + c.L - sp.q0;
    d = d >= c.L ? d - c.L : d;
    return d < sp.k;
}

// Wave wv of NSEL clears its share of the deposit (o, y, x): phase one cuts
// the lines (the selecting wave also the deposit's own line), phase two
// turns the block's cuts into row counts; the selecting waves meet between.
template <int NSEL>
__device__ __forceinline__ void interval_clear(const Ctx &c, uint32_t o, uint32_t y, uint32_t x, uint32_t t,
                                               uint32_t wv, uint32_t &wchg, uint64_t &occ, uint32_t &passed,
                                               unsigned long long *acc = nullptr)
{
    uint64_t pt = acc ? tick() : 0;
    const uint32_t L = c.L, k = c.k, lane = lane_id();
    const uint32_t strip = 2 * k - 1 < L ? 2 * k - 1 : L;
    // this step's difference counts
    uint32_t *const dD = c.dD + (t & 1u) * c.ivstride;
    uint32_t *const dC = dD + interval_diff_words(k);
    uint32_t xb = x + L - (k - 1);
    xb = xb >= L ? xb - L : xb;
    uint32_t yb = y + L - (k - 1);
    yb = yb >= L ? yb - L : yb;
    bool bad = false;
    // ---- phase one: every read of this wave's share is issued first, so the
    // share costs one round trip; the occupancy hash of the deposit's sites
    // (split over the waves) runs while the reads are in flight
    // the deposit's own line (selecting wave, one lane): H row y loses
    // [x-k+1, x+k-1], V column x loses [y-k+1, y+k-1]
    uint32_t *const slist = o ? c.vb : c.hb;
    const uint32_t sq = o ? x : y;
    const CutPlan spl = cut_plan(c, o ? yb : xb, strip);
    const bool sact = wv == 0 && lane == 0;
    // the crossing lines: for H, V columns x .. x+k-1 lose rows [y-k+1, y];
    // for V, H rows y .. y+k-1 lose columns [x-k+1, x]; 64-line blocks
    // round-robin over the waves, up to IV_PF of them read at once
    constexpr int IV_PF = 4;
    const Span sp = make_span(c, o ? y : x, k);
    uint32_t *const blist = o ? c.hb : c.vb;
    const uint32_t blo = o ? xb : yb;
    const CutPlan bp = cut_plan(c, blo, k);
    // Every read of a pass is issued before any is used.  The first pass is
    // written out of the loop, and the deposit's own line is read after its
    // block reads: a wait for that read placed ahead of them (the compiler
    // moves the own line's arithmetic up) would cost a second round trip.
    uint32_t ev[IV_PF][4];
    uint32_t qv[IV_PF];
    bool av[IV_PF];
    const auto prefetch = [&](uint32_t m0) {
#pragma unroll
        for (int f = 0; f < IV_PF; ++f) {
            const uint32_t m = m0 + (uint32_t)f * NSEL;
            const uint32_t q = m < sp.n ? span_block(sp, m) * 64 + lane : 0xFFFFFFFFu;
            av[f] = m < sp.n && in_span(c, sp, q);
            qv[f] = q;
            cut_load(c, bp, blist, q, av[f], ev[f]);
        }
    };
    const auto apply = [&](uint32_t m0) {
#pragma unroll
        for (int f = 0; f < IV_PF; ++f) {
            const uint32_t m = m0 + (uint32_t)f * NSEL;
            if (m >= sp.n) break;
            const uint32_t blk = span_block(sp, m);
            const uint32_t q = qv[f];
            const bool act = av[f];
            const LineCut cut = cut_apply(c, bp, blist, q, act, ev[f]);
            bad = bad || cut.bad;
            if (o == 1) {
                // H row q: its count drops by the anchors removed
                count_sub_wave(c, act, q, cut.n);
                wchg += cut.nw;
                continue;
            }
            // V column q: rows blo + [l, h] (block-relative) lose an anchor
            const bool has = act && cut.n != 0;
            uint32_t l = 0;
            if (has && cut.n < k) {
                l = cut.start + L - blo;
                l = l >= L ? l - L : l;
            }
            const uint32_t h = l + cut.n - 1;
            // a cut lies inside the block's k rows; anything else is a broken
            // invariant and is reported, never written
            const bool in_block = h < k;
            bad = bad || (has && !in_block);
            const bool has_ok = has && in_block;
            if (has_ok) {
                atomicAdd(&dD[l], 1u);
                atomicAdd(&dC[l >> 6], 1u);
                if (h + 1 < k) {
                    atomicSub(&dD[h + 1], 1u);
                    atomicSub(&dC[(h + 1) >> 6], 1u);
                }
            }
            // the row-major V bitmap: word blk of every row where some column
            // of it lost an anchor; the span's bits of it become 0.  Lane j
            // writes rows g*64 + j (block-relative) for the 64-row groups g
            // in its mask, built from the block's distinct cut ranges
            uint64_t pend = __ballot(has_ok);
            if (pend == 0) continue;
            const uint64_t spanmask = __ballot(act);
            const bool whole = spanmask == ~0ull;
            uint64_t M = 0;
            uint32_t glo_all = 64, ghi_all = 0;
            while (pend) {
                const uint32_t f = first_lane(pend);
                const uint32_t lf = bcast(l, f), hf = bcast(h, f);
                pend &= ~__ballot(has_ok && l == lf && h == hf);
                // group g holds row g*64 + lane inside [lf, hf] for
                // ceil((lf - lane) / 64) <= g <= floor((hf - lane) / 64)
                const int32_t a = ((int32_t)lf - (int32_t)lane + 63) >> 6;
                const int32_t b = ((int32_t)hf - (int32_t)lane) >> 6;
                M |= bit_range(a, b);
                glo_all = min(glo_all, lf >> 6);
                ghi_all = max(ghi_all, hf >> 6);
            }
            wchg += (uint32_t)__popcll(M);
            uint64_t *const bm = c.av1;
            for (uint32_t g = glo_all; g <= ghi_all; ++g) {
                if ((M >> g) & 1ull) {
                    uint32_t row = blo + g * 64 + lane;
                    row = row >= L ? row - L : row;
                    const uint32_t at = bm_index(c, row, blk);
                    if (whole)
                        gst64(&bm[at], 0ull);
                    else
                        gand64(&bm[at], ~spanmask);
                }
            }
        }
    };
    // shares: block m goes to wave (m + 1) % NSEL, so the selecting wave, which
    // also cuts the deposit's own line, has the fewest blocks
    const uint32_t w0 = (wv + NSEL - 1) % NSEL;
    prefetch(w0);
    uint32_t sev[4];
    cut_load(c, spl, slist, sq, sact, sev);
    // this wave's share of the occupancy hash: site i of the deposit
    for (uint32_t i = w0 * 64 + lane; i < k; i += NSEL * 64) {
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
    if (wv == 0) {
        const LineCut cut = cut_apply(c, spl, slist, sq, sact, sev);
        bad = bad || cut.bad;
        if (lane == 0) {
            if (o == 0) {
                if (cut.n) count_sub(c, y, cut.n);
                wchg += cut.nw;
            } else {
                c.h->jrs = cut.start;
                c.h->jn = cut.n;
                wchg += cut.n;   // one V word per row of the column
            }
        }
    }
    apply(w0);
    for (uint32_t m0 = w0 + NSEL * IV_PF; m0 < sp.n; m0 += NSEL * IV_PF) {
        prefetch(m0);
        apply(m0);
    }
    if (__ballot(bad) && lane == 0) c.h->status = kErrSelect;
    if (acc) {
        const uint64_t t1 = tick();
        if (lane == 0) acc[kAccIvCut] += t1 - pt;
        pt = t1;
    }
    // counts in the slab: this wave's atomics (and its clearing of the set
    // two steps back) are done at L2 before the waves meet
    if (c.ivg) __builtin_amdgcn_s_waitcnt(0);
    sel_barrier<NSEL>(c, passed, wv == 0);
    if (acc) {
        const uint64_t t1 = tick();
        if (lane == 0) acc[kAccIvMeet] += t1 - pt;
        pt = t1;
    }
    // ---- phase two
    if (o == 0) {
        // V rows blo + i, i < k: the counts drop by the number of columns
        // whose cut covers row i (difference counts, their 64-row sums give
        // each block's carry)
        const uint32_t nC = (k + 63) >> 6;   // <= 64
        const auto row_group = [&](uint32_t m, uint32_t dv, uint32_t cex) {
            const uint32_t i = m * 64 + lane;
            const bool act = i < k;
            if (act) dD[i] = 0u;
            const uint32_t dcount = wave_scan(act ? dv : 0u) + bcast(cex, m);
            uint32_t row = blo + i;
            row = row >= L ? row - L : row;
            count_sub_wave(c, act, L + row, dcount);
        };
        if (!c.ivg) {
            const uint32_t cv = lane < nC ? lds_peek(&dC[lane]) : 0u;
            const uint32_t cex = wave_scan(cv) - cv;
            for (uint32_t m = w0; m < nC; m += NSEL) {
                const uint32_t i = m * 64 + lane;
                row_group(m, i < k ? lds_peek(&dD[i]) : 0u, cex);
            }
        } else {
            // counts in the slab: up to 8 of the wave's row groups read at
            // once (every lane reads an entry that exists; out-of-range ones
            // are masked where they are used)
            const auto ld = [](const uint32_t *p) {
                return __hip_atomic_load((const gmem<uint32_t> *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            };
            const uint32_t cv0 = ld(&dC[lane]);
            const uint32_t cv = lane < nC ? cv0 : 0u;
            const uint32_t cex = wave_scan(cv) - cv;
            for (uint32_t m0 = w0; m0 < nC; m0 += 8 * NSEL) {
                uint32_t dv[8];
#pragma unroll
                for (uint32_t u = 0; u < 8; ++u) {
                    const uint32_t i = (m0 + u * NSEL) * 64 + lane;
                    dv[u] = ld(&dD[i < k ? i : 0u]);
                }
#pragma unroll
                for (uint32_t u = 0; u < 8; ++u) {
                    const uint32_t m = m0 + u * NSEL;
                    if (m >= nC) break;
                    row_group(m, dv[u], cex);
                }
            }
        }
    } else {
        // V rows of the deposit's own column that lost their anchor at x
        const uint32_t jrs = lds_peek(&c.h->jrs), jn = lds_peek(&c.h->jn);
        uint64_t *const bm = c.av1;
        const uint64_t bit = 1ull << (x & 63u);
        for (uint32_t m = w0; m * 64 < jn; m += NSEL) {
            const uint32_t i = m * 64 + lane;
            const bool act = i < jn;
            uint32_t row = jrs + i;
            row = row >= L ? row - L : row;
            count_sub_wave(c, act, L + row, 1u);
            if (act) gand64(&bm[bm_index(c, row, x >> 6)], ~bit);
        }
    }
    if (acc && lane == 0) acc[kAccIvRows] += tick() - pt;
}

// Words a lane holds of one bitmap row: lane, lane+64, ... (ROWW of them;
// ROWW = 1 covers L <= 4096, 8 covers L <= 32768).
template <int ROWW>
struct RowWords {
    uint64_t w[ROWW];
};

template <int ROWW>
__device__ __forceinline__ void load_row(const Ctx &c, uint32_t R, RowWords<ROWW> &rw)
{
    const uint32_t lane = lane_id();
    const uint32_t o = R >= c.L ? 1u : 0u, y = R - o * c.L;
    const uint64_t *bm = bitmap(c, o);
    const uint32_t per = (c.wd + 63) >> 6;
#pragma unroll
    for (uint32_t j = 0; j < ROWW; ++j) {
        uint32_t wi = lane + 64 * j;
        rw.w[j] = (j < per && wi < c.wd) ? bm[bm_index(c, y, wi)] : 0;
    }
}

// Apply a clear to row words read before it (the clear only ever removes
// bits inside its masks, so this gives the row as it is after the clear).
template <int ROWW>
__device__ __forceinline__ void patch_rect(const Ctx &c, const Rect &r, uint32_t o, uint32_t y,
                                           RowWords<ROWW> &rw)
{
    const uint32_t lane = lane_id();
    const uint32_t L = c.L;
    uint32_t dy = y + L - r.row0;
    dy = dy >= L ? dy - L : dy;
    if (r.o != o || dy >= r.nrows) return;
    const uint32_t per = (c.wd + 63) >> 6;
#pragma unroll
    for (uint32_t j = 0; j < ROWW; ++j) {
        uint32_t wi = lane + 64 * j;
        if (j < per && wi < c.wd) rw.w[j] &= ~col_mask(L, r.c0, r.len, wi);
    }
}

template <int ROWW>
__device__ __forceinline__ void patch_row(const Ctx &c, const Clear &cl, uint32_t R, RowWords<ROWW> &rw)
{
    const uint32_t o = R >= c.L ? 1u : 0u, y = R - o * c.L;
    patch_rect(c, cl.a, o, y, rw);
    patch_rect(c, cl.b, o, y, rw);
}

// Hierarchical select on the LDS counts: the row R holding the available
// placement of rank r (r < A) and r's offset inside that row.  `inc2` and
// `v2` are this lane's inclusive scan and value over the 4096-row sums.
__device__ __forceinline__ bool locate_row(const Ctx &c, uint32_t inc2, uint32_t v2, uint32_t r,
                                           uint32_t &R, uint32_t &rin)
{
    const uint32_t lane = lane_id();
    uint32_t g = 0;
    if (c.n2() > 1) {
        uint64_t bal = __ballot(inc2 > r);
        if (bal == 0) return false;
        g = first_lane(bal);
        r -= bcast(inc2 - v2, g);
    }
    uint32_t i1 = g * 64 + lane;
    uint32_t v = i1 < c.n1() ? lds_peek(&c.cnt1[i1]) : 0;
    uint32_t inc = wave_scan(v);
    uint64_t bal = __ballot(inc > r);
    if (bal == 0) return false;
    uint32_t l1 = first_lane(bal);
    r -= bcast(inc - v, l1);
    g = g * 64 + l1;
    uint32_t i0 = g * 64 + lane;
    v = i0 < 2 * c.L ? row_count(c, i0) : 0;
    inc = wave_scan(v);
    bal = __ballot(inc > r);
    if (bal == 0) return false;
    uint32_t l0 = first_lane(bal);
    r -= bcast(inc - v, l0);
    R = uniform(g * 64 + l0);
    rin = uniform(r);
    return R < 2 * c.L;
}

// Position of the r-th (0-based) set bit of w, by halving with popcounts;
// 64 + something when w has no more than r set bits.
__device__ __forceinline__ uint32_t select_bit(uint64_t w, uint32_t r)
{
    const uint32_t n = (uint32_t)__popcll(w);
    uint32_t pos = r < n ? 0u : 64u;
    uint32_t c = (uint32_t)__popc((uint32_t)w);
    uint32_t v = (uint32_t)w;
    if (r >= c) {
        r -= c;
        v = (uint32_t)(w >> 32);
        pos += 32;
    }
#pragma unroll
    for (uint32_t half = 16; half >= 1; half >>= 1) {
        c = (uint32_t)__popc(v & ((1u << half) - 1));
        if (r >= c) {
            r -= c;
            v >>= half;
            pos += half;
        }
    }
    return pos;
}

// The rin-th available placement of row R: canonical index, or false.  Each
// lane selects the bit its own residual rank points at while the wave finds
// the lane that holds the placement; that lane's answer is read last.
template <int ROWW>
__device__ __forceinline__ bool pick_in_row(const Ctx &c, const RowWords<ROWW> &rw, uint32_t R, uint32_t rin,
                                            uint32_t &P)
{
    const uint32_t per = (c.wd + 63) >> 6;
    uint32_t x = 0xFFFFFFFFu;
    bool found = false;
#pragma unroll
    for (uint32_t j = 0; j < ROWW; ++j) {
        if (!found && j < per) {
            const uint32_t pc = (uint32_t)__popcll(rw.w[j]);
            const uint32_t pinc = wave_scan(pc);
            const uint32_t tot = bcast(pinc, 63);
            if (rin < tot) {
                const uint32_t mine = select_bit(rw.w[j], rin - (pinc - pc));
                const uint32_t l = first_lane(__ballot(pinc > rin));
                const uint32_t pos = bcast(mine, l);
                if (pos < 64) x = (l + 64 * j) * 64 + pos;
                found = true;
            } else {
                rin -= tot;
            }
        }
    }
    if (x >= c.L) return false;
    const uint32_t o = R >= c.L ? 1u : 0u;
    P = uniform(o * c.L2() + (R - o * c.L) * c.L + x);
    return true;
}

// Scan of the 4096-row sums: A_t, and this lane's scan value.
__device__ __forceinline__ uint32_t scan_top(const Ctx &c, uint32_t &inc2, uint32_t &v2)
{
    const uint32_t lane = lane_id();
    if (c.n2() == 1) {   // one group: its sum is A, no scan needed
        v2 = lds_peek(&c.cnt2[0]);
        inc2 = v2;
        return uniform(v2);
    }
    v2 = lane < c.n2() ? lds_peek(&c.cnt2[lane]) : 0;
    inc2 = wave_scan(v2);
    return bcast(inc2, 63);
}

// Rows y0 .. y0+nr-1 of bitmap o read ahead of a clear, flattened: word q =
// (row - y0) * wd + w is held by lane q % 64 in slot q / 64.
template <int SPW>
struct SpecRows {
    uint64_t w[SPW];
    uint32_t o, y0, nr;
};

// Where to read ahead: the rows where the next placement is expected once
// the clear `cl` has landed.  The next rank lies near u*(A - C)/2^64, and in
// the counts before the clear up to C further on, where C is the number of
// placements the clear removes; C is estimated as the rectangles' area times
// the available fraction A / 2L^2, and the window is centred half-way.  LDS
// only, so it can run while the clear's reads are in flight.
template <int SPW>
__device__ __forceinline__ void plan_ahead(const Ctx &c, const Clear &cl, uint64_t u, float inv2l2,
                                           SpecRows<SPW> &sp)
{
    const uint32_t L = c.L;
    sp.o = sp.y0 = sp.nr = 0;
    uint32_t inc2, v2, R, rin;
    const uint32_t A = scan_top(c, inc2, v2);
    if (A <= 1) return;
    const float area = (float)cl.a.nrows * (float)cl.a.len + (float)cl.b.nrows * (float)cl.b.len;
    uint32_t C = uniform((uint32_t)(area * ((float)A * inv2l2)));
    C = C < A ? C : A - 1;
    const uint32_t r = draw_rank(u, A - C) + C / 2;
    if (!locate_row(c, inc2, v2, r < A ? r : A - 1, R, rin)) return;
    const uint32_t o = R >= L ? 1u : 0u, y = R - o * L;
    const uint32_t nr = c.spec_rows < L ? c.spec_rows : L;
    uint32_t y0 = y >= nr / 2 ? y - nr / 2 : 0;
    y0 = y0 + nr > L ? L - nr : y0;
    sp.o = o;
    sp.y0 = y0;
    sp.nr = nr;
}

// Issue the reads of the planned window, without branches (a lane past the
// window reads the window's first word and never hands it on), so that the
// compiler keeps them in flight until the select takes a row from them.  A
// word may be read before or after the clear (or a helper wave's share of
// it) has written it: the select patches the window with the clear's masks,
// so either value serves.
template <int SPW>
__device__ __forceinline__ void load_ahead(const Ctx &c, SpecRows<SPW> &sp)
{
    const uint32_t lane = lane_id(), wd = c.wd;
    const gmem<uint64_t> *bm = (const gmem<uint64_t> *)bitmap(c, sp.o);
    const uint32_t nq = sp.nr * wd;
#pragma unroll
    for (int j = 0; j < SPW; ++j) {
        const uint32_t q0 = lane + 64 * j;
        const uint32_t q = q0 < nq ? q0 : 0;   // in bounds: row y0 < L, word 0
        const uint32_t dr = fdiv(q, c.fwd);
        const uint64_t v = bm[bm_index(c, sp.y0 + dr, q - dr * wd)];
        sp.w[j] = v;   // words past the window are never taken from it
    }
}

// Row R out of the read-ahead window (the caller checked it is inside).
template <int SPW, int ROWW>
__device__ __forceinline__ void row_from_window(const Ctx &c, const SpecRows<SPW> &sp, uint32_t y,
                                                RowWords<ROWW> &rw)
{
    const uint32_t lane = lane_id(), wd = c.wd;
#pragma unroll
    for (int j = 0; j < ROWW; ++j) {
        uint32_t w = lane + 64 * j;
        uint32_t q = (y - sp.y0) * wd + w;
        uint32_t src = q & 63, slot = q >> 6;
        uint64_t val = 0;
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            uint64_t v = __shfl(sp.w[s], src, 64);
            if (slot == (uint32_t)s) val = v;
        }
        rw.w[j] = w < wd ? val : 0;
    }
}

// The rin-th available placement of row R (canonical index in P): for H
// rows under the interval clear from the row's buckets (one entry per lane,
// in position order), otherwise from the row's bitmap words.
template <int ROWW>
__device__ __forceinline__ bool pick_row(const Ctx &c, uint32_t R, uint32_t rin, uint32_t &P)
{
    if (c.interval && R < c.L) {
        const uint32_t lane = lane_id();
        const uint32_t nS = num_buckets(c.L, c.k);
        const uint32_t E = lane < nS ? gld32(&c.hb[lane * c.lp() + R]) : kNoSeg;
        const uint32_t len = E == kNoSeg ? 0u : seg_end(E) - seg_start(E) + 1;
        const uint32_t inc = wave_scan(len);
        const uint64_t bal = __ballot(inc > rin);
        if (bal == 0) return false;
        const uint32_t j = first_lane(bal);
        const uint32_t x = bcast(seg_start(E), j) + (rin - bcast(inc - len, j));
        if (x >= c.L) return false;
        P = uniform(R * c.L + x);
        return true;
    }
    RowWords<ROWW> rw;
    load_row(c, R, rw);
    return pick_in_row(c, rw, R, rin, P);
}

template <int NSEL>
struct TileCap {
    static constexpr int value = NSEL == 1 ? 4 : 8;
};

// ---------------------------------------------------------------------------
// Selecting wave
// ---------------------------------------------------------------------------

// deadline: wall-clock tick at which the run yields (0 = run to jamming); it
// is checked every 16 steps, at a step whose placement is selected but not
// yet deposited, so the saved state resumes exactly there.
template <int NSEL, int ROWW, bool SPARSE, bool STOP>
__device__ __forceinline__ void selector(Ctx &c, uint64_t deadline)
{
    constexpr int CAP = TileCap<NSEL>::value;
    // read-ahead window (words per lane); for rows wider than 64 words the
    // window covers too few rows to hit often, so it is left out
    constexpr int SPW = ROWW == 1 ? 2 : 0;
    const uint32_t lane = lane_id();
    __builtin_amdgcn_s_setprio(3);   // latency-critical chain first on a shared SIMD
    const uint32_t L = c.L, k = c.k;
    const uint32_t t_begin = c.h->t0;
    // with STOP, selection ends before step h->stop as if the lattice jammed there
    const uint32_t stop_at = STOP && c.h->stop ? c.h->stop : 0xFFFFFFFFu;
    uint64_t occ = 0, seqh = c.h->seqh;
    uint32_t wchg = 0;
    const bool prof = c.prof != nullptr;
    unsigned long long *const acc = c.h->sel_acc;   // lane 0 adds to these when profiling
    const float inv2l2 = 1.0f / (2.0f * (float)L * (float)L);   // read-ahead estimate only
    uint64_t p0 = 0;
    if (prof && lane == 0) acc[kAccStart] = tick();
    // draws for the 64 steps of t_begin's block (lane = step within the block)
    uint64_t u_pre = philox_u64((t_begin & ~63u) + lane, c.sample, c.k0, c.k1);
    uint32_t t = t_begin;
    uint32_t P = c.h->p0;
    bool alive = true, yielded = false;
    uint32_t passed = 0;   // mid-step barriers of the interval clear
    if (!c.h->resumed) {   // first placement
        uint32_t inc2, v2, R, rin;
        uint32_t A = scan_top(c, inc2, v2);
        uint32_t r = uniform(draw_rank(bcast64(u_pre, 0), A));
        alive = A > 0 && locate_row(c, inc2, v2, r, R, rin);
        if (alive) alive = pick_row<ROWW>(c, R, rin, P);
        if (!alive && A > 0 && lane == 0) c.h->status = kErrSelect;
    }
    while (alive) {
        // ---- step t: P is known.
        if (STOP && t == stop_at) break;
        if (deadline && (t & 15) == 0 && t != t_begin && tick() >= deadline) {
            yielded = true;
            break;
        }
        // A correct run never deposits more than L*L/k k-mers; stop before
        // the k-mer records would overflow.
        if (t + 1 >= c.ncap) {
            if (lane == 0) c.h->status = kErrSelect;
            break;
        }
        // every 64 steps: wait for ring room for the next 64 placements
        if ((t & 63) == 0 && t + 64 > kRing) {
            if (prof) p0 = tick();
            while (!lds_load(&c.h->lab_exit) && t + 64 - lds_load(&c.h->lab_progress) > kRing)
                __builtin_amdgcn_s_sleep(2);
            if (prof && lane == 0) acc[kAccRing] += tick() - p0;
        }
        if (prof) p0 = tick();
        if (lane == 0) {
            c.ring[t & (kRing - 1)] = P;
            lds_store(&c.h->sel_progress, t + 1);
        }
        const uint32_t o = P >= c.L2() ? 1u : 0u;
        const uint32_t rem = P - o * c.L2();
        const uint32_t y = fdiv(rem, c.fL), x = rem - y * L;
        const Clear cl = make_clear(c, o, y, x);
        if (NSEL > 1 && lane == 0) {
            c.h->cur_p = P;
            lds_store(&c.h->clr_gen, t + 1);
        }
        // draw for step t+1
        const uint32_t t1 = t + 1;
        if ((t1 & 63) == 0) u_pre = philox_u64(t1 + lane, c.sample, c.k0, c.k1);
        const uint64_t u1 = bcast64(u_pre, t1 & 63);
        // hashes of the deposit: pure arithmetic, run while the clear's
        // reads are in flight
        const auto hash_step = [&] {
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
        };
        // The rows where step t+1 will most likely pick are read ahead.
        // Dense clear: the window is planned (LDS scans) while the clear's
        // reads are in flight and read as soon as they have landed, so its
        // reads overlap the clear's writes and the exact select's scans.
        // Sparse clear: planned and read first, then the clear's dependent
        // round trips cover the window's.
        SpecRows<SPW == 0 ? 1 : SPW> sp;
        sp.o = sp.y0 = sp.nr = 0;
        uint64_t ph = prof ? tick() : 0;
        if constexpr (SPARSE) {
            if (c.interval) {
                seqh += mix64(((uint64_t)t << 32) | P);   // the sites' hash is split over the waves
                interval_clear<NSEL>(c, o, y, x, t, 0, wchg, occ, passed, prof ? acc : nullptr);
                if (prof && lane == 0) acc[kAccProcess] += tick() - ph;
            } else {
                if constexpr (SPW > 0) {
                    plan_ahead<SPW>(c, cl, u1, inv2l2, sp);
                    load_ahead<SPW>(c, sp);
                }
                if (prof) {
                    uint64_t ph1 = tick();
                    if (lane == 0) acc[kAccHook] += ph1 - ph;
                    ph = ph1;
                }
                hash_step();
                sparse_clear<CAP>(c, cl, 0, NSEL, wchg);
                if (prof && lane == 0) acc[kAccProcess] += tick() - ph;
            }
        } else {
            const auto hook = [&] {
                hash_step();
                if constexpr (SPW > 0) plan_ahead<SPW>(c, cl, u1, inv2l2, sp);
            };
            const auto landed = [&] {
                if constexpr (SPW > 0) load_ahead<SPW>(c, sp);
            };
            clear_items<CAP, ROWW == 1>(c, cl, 0, NSEL, wchg, hook, landed);
            if (prof && lane == 0) acc[kAccProcess] += tick() - ph;
        }
        if (NSEL > 1) {
            // helpers' bitmap stores must be visible before the next select
            uint32_t want = t1 * (NSEL - 1);
            __builtin_amdgcn_s_setprio(0);
            while (lds_load(&c.h->clr_done) < want) __builtin_amdgcn_s_sleep(1);
            __builtin_amdgcn_s_setprio(3);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        if (SPARSE && c.interval && o == 0) {
            // every wave is past this step's block sums: clear them for the
            // next use of this set
            if (lane < ((k + 63) >> 6)) c.dC[(t & 1u) * c.ivstride + lane] = 0u;
        }
        if (prof) {
            uint64_t p1 = tick();
            if (lane == 0) acc[kAccClear] += p1 - p0;
            p0 = p1;
        }
        // ---- exact select for step t+1
        t = t1;
        uint32_t inc2, v2, R, rin;
        const uint32_t A = scan_top(c, inc2, v2);
        if (A == 0) break;
        if (!locate_row(c, inc2, v2, draw_rank(u1, A), R, rin)) {
            if (lane == 0) c.h->status = kErrSelect;
            break;
        }
        if (SPARSE && c.interval) {
            if (!pick_row<ROWW>(c, R, rin, P)) {
                if (lane == 0) c.h->status = kErrSelect;
                break;
            }
        } else {
            RowWords<ROWW> rw;
            const uint32_t ro = R >= L ? 1u : 0u, ry = R - ro * L;
            if (SPW > 0 && sp.nr && ro == sp.o && ry >= sp.y0 && ry < sp.y0 + sp.nr) {
                row_from_window<SPW == 0 ? 1 : SPW, ROWW>(c, sp, ry, rw);
                patch_row(c, cl, R, rw);
                if (prof && lane == 0) ++acc[kAccSpec];
            } else {
                load_row(c, R, rw);
            }
            if (!pick_in_row(c, rw, R, rin, P)) {
                if (lane == 0) c.h->status = kErrSelect;
                break;
            }
        }
        if (prof && lane == 0) acc[kAccSelect] += tick() - p0;
    }
    if (prof) {
        prof_add(c, kProfSelTotal, tick() - acc[kAccStart]);
        prof_add(c, kProfSelRing, acc[kAccRing]);
        prof_add(c, kProfSelSelect, acc[kAccSelect]);
        prof_add(c, kProfSelClear, acc[kAccClear]);
        prof_add(c, kProfSteps, t);
        prof_add(c, kProfSpecHits, acc[kAccSpec]);
        prof_add(c, kProfSelHook, acc[kAccHook]);
        prof_add(c, kProfSelProcess, acc[kAccProcess]);
        prof_add(c, kProfIvCut, acc[kAccIvCut]);
        prof_add(c, kProfIvMeet, acc[kAccIvMeet]);
        prof_add(c, kProfIvRows, acc[kAccIvRows]);
    }
    occ = wave_sum64(occ);
    uint32_t wsum = wave_sum32(wchg);
    if (lane == 0) {
        atomicAdd(&c.h->occ, (unsigned long long)occ);
        atomicAdd(&c.h->wchg, (unsigned long long)wsum);
        c.h->seqh = seqh;
        if (yielded) {
            c.h->p0 = P;
            c.h->preempt = 1;
        }
        lds_store(&c.h->sel_done, t + 1);
    }
}

template <int NSEL, int ROWW, bool SPARSE>
__device__ __forceinline__ void helper(Ctx &c, uint32_t wv)
{
    constexpr int CAP = TileCap<NSEL>::value;
    const uint32_t lane = lane_id();
    __builtin_amdgcn_s_setprio(2);
    uint32_t wchg = 0;
    uint64_t occ = 0;       // this wave's share of the occupancy hash (interval clear)
    uint32_t passed = 0;    // mid-step barriers of the interval clear
    uint32_t g = c.h->t0;   // clear requests are numbered by step
    for (;;) {
        uint32_t gen;
        bool stop = false;
        // waiting for the next clear: the selecting wave's select goes first
        __builtin_amdgcn_s_setprio(0);
        for (;;) {
            gen = lds_load(&c.h->clr_gen);
            if (gen > g) break;
            if (lds_load(&c.h->sel_done)) {
                stop = true;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_s_setprio(2);
        if (stop) break;
        g = gen;
        uint32_t P = uniform(lds_peek(&c.h->cur_p));
        uint32_t o = P >= c.L2() ? 1u : 0u;
        uint32_t rem = P - o * c.L2();
        uint32_t y = fdiv(rem, c.fL);
        uint32_t x = rem - y * c.L;
        if constexpr (SPARSE) {
            if (c.interval)
                interval_clear<NSEL>(c, o, y, x, g - 1, wv, wchg, occ, passed);
            else
                sparse_clear<CAP>(c, make_clear(c, o, y, x), wv, NSEL, wchg);
        } else {
            clear_items<CAP, ROWW == 1>(c, make_clear(c, o, y, x), wv, NSEL, wchg);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) atomicAdd(&c.h->clr_done, 1u);
    }
    uint32_t wsum = wave_sum32(wchg);
    occ = wave_sum64(occ);
    if (lane == 0) {
        atomicAdd(&c.h->wchg, (unsigned long long)wsum);
        if (occ) atomicAdd(&c.h->occ, (unsigned long long)occ);
    }
}

// ---------------------------------------------------------------------------
// Compressed lattice (long k-mers)
// ---------------------------------------------------------------------------
// A site keeps one bit in each of: occupied by an H k-mer, by a V k-mer, H
// anchor, V anchor (the parent site of Sec. II.E).  The labelling wave needs,
// for every contact of a new k-mer, the k-mer on the other side: a k-mer that
// crosses the new one's side line ends or starts right there (it cannot
// reach the new k-mer's sites), so its anchor is known outright; one lying
// along the side line is found from the anchor bits, its first contact at an
// anchor or at the side's first site (there by the nearest anchor before
// it); a k-mer met at an end of the new one is either of these.  The
// canonical placement index of that anchor gives the deposit number through
// an open-addressing table written as k-mers are labelled.  Occupancies are
// read along rows (H deposits' sides) and along columns (V deposits'); a
// copy written across its lines is tiled 16 lines to a 128-byte tile so the
// k bits a deposit sets there touch k/16 lines.  Bitmap words and table
// slots are changed by atomics at L2 and read with L2-scope loads.

__device__ __forceinline__ uint32_t word_plain(const Ctx &c, uint32_t line, uint32_t w) { return line * c.nlw + w; }
__device__ __forceinline__ uint32_t word_tiled(const Ctx &c, uint32_t line, uint32_t w)
{
    return ((w * c.nt16 + (line >> 4)) << 4) + (line & 15u);
}

__device__ __forceinline__ uint64_t ld_l2(const uint64_t *p)
{
    return __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void or_l2(uint64_t *p, uint64_t m)
{
    if (m) atomicOr((unsigned long long *)p, (unsigned long long)m);
}

// Bit `pos` along line `line` of a bitmap (plain or tiled).
__device__ __forceinline__ uint32_t bit_plain(const Ctx &c, const uint64_t *bm, uint32_t line, uint32_t pos)
{
    return (uint32_t)(ld_l2(&bm[word_plain(c, line, pos >> 6)]) >> (pos & 63u)) & 1u;
}
__device__ __forceinline__ uint32_t bit_tiled(const Ctx &c, const uint64_t *bm, uint32_t line, uint32_t pos)
{
    return (uint32_t)(ld_l2(&bm[word_tiled(c, line, pos >> 6)]) >> (pos & 63u)) & 1u;
}

// Placement -> deposit number: slots of (P + 1) | t << 32, linear probing
// from a multiplicative hash.
__device__ __forceinline__ uint32_t kh_slot(const Ctx &c, uint32_t P)
{
    return (uint32_t)((P * 0x9E3779B1u) >> (32 - c.hlg));
}

__device__ __forceinline__ void kh_insert(const Ctx &c, uint32_t P, uint32_t t)
{
    const uint32_t mask = (1u << c.hlg) - 1;
    uint32_t sl = kh_slot(c, P);
    const unsigned long long v = (unsigned long long)(P + 1) | ((unsigned long long)t << 32);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        if (atomicCAS(&c.khash[sl], 0ull, v) == 0ull) return;
        sl = (sl + 1) & mask;
    }
}

// Deposit number of the k-mer placed at P, or -1 if the table has none.
__device__ __forceinline__ int32_t kh_find(const Ctx &c, uint32_t P)
{
    const uint32_t mask = (1u << c.hlg) - 1;
    uint32_t sl = kh_slot(c, P);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const unsigned long long e =
            __hip_atomic_load(&c.khash[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)e == P + 1) return (int32_t)(e >> 32);
        if (e == 0ull) return -1;
        sl = (sl + 1) & mask;
    }
    return -1;
}

// Set bits [a, a + len) (cyclic, len <= L) along line `line` of a plain
// bitmap: the wave's lanes take one word each.
__device__ __forceinline__ void set_run_plain(const Ctx &c, uint64_t *bm, uint32_t line, uint32_t a, uint32_t len)
{
    const uint32_t L = c.L, lane = lane_id();
    const uint32_t e1 = a + len < L ? a + len : L;   // [a, e1) then [0, a + len - L)
    const uint32_t n1 = ((e1 - 1) >> 6) - (a >> 6) + 1;
    const uint32_t e2 = a + len > L ? a + len - L : 0;
    const uint32_t n2 = e2 ? ((e2 - 1) >> 6) + 1 : 0;
    for (uint32_t i = lane; i < n1 + n2; i += 64) {
        uint32_t w, lo, hi;   // word and the run's positions in it, [lo, hi)
        if (i < n1) {
            w = (a >> 6) + i;
            lo = w * 64 > a ? w * 64 : a;
            hi = w * 64 + 64 < e1 ? w * 64 + 64 : e1;
        } else {
            w = i - n1;
            lo = w * 64;
            hi = w * 64 + 64 < e2 ? w * 64 + 64 : e2;
        }
        or_l2(&bm[word_plain(c, line, w)], bit_range((int32_t)(lo - w * 64), (int32_t)(hi - w * 64) - 1));
    }
}

// Nearest set bit at or before position p, cyclically, within distance d
// (positions p - d .. p) along line `line` of a plain bitmap; ~0u if none.
// All lanes of the wave take part.
__device__ __forceinline__ uint32_t nearest_before(const Ctx &c, const uint64_t *bm, uint32_t line, uint32_t p,
                                                   uint32_t d)
{
    const uint32_t L = c.L, lane = lane_id(), nw = c.nlw;
    const uint32_t pw = p >> 6;
    // words pw, pw - 1, ... back round the line (one more than full words
    // would need: crossing the seam passes the line's short last word); the
    // last step (back at pw) holds the positions after p, reached only when
    // d spans almost all of L
    uint32_t steps = (d + 63) / 64 + 2;
    steps = steps < nw ? steps : nw;
    const bool wrapback = d + 64 >= L;
    const uint32_t total = steps + (wrapback ? 1u : 0u);
    for (uint32_t l0 = 0; l0 < total; l0 += 64) {
        const uint32_t l = l0 + lane;
        uint32_t cand = ~0u;
        if (l < total) {
            const bool again = wrapback && l == total - 1;   // pw's positions after p
            uint32_t w = again ? pw : (pw + nw * 2 - (l % nw)) % nw;
            const uint32_t valid = w == nw - 1 && (L & 63u) ? (L & 63u) : 64u;
            uint64_t m = ld_l2(&bm[word_plain(c, line, w)]) & (valid == 64 ? ~0ull : ((1ull << valid) - 1));
            if (!again && l == 0) m &= bit_range(0, (int32_t)(p & 63u));
            if (again) m &= ~bit_range(0, (int32_t)(p & 63u));
            if (m) {
                const uint32_t q = w * 64 + (63 - __clzll((long long)m));
                const uint32_t dist = p >= q ? p - q : p + L - q;
                if (dist <= d) cand = q;
            }
        }
        const uint64_t hit = __ballot(cand != ~0u);
        if (hit) return bcast(cand, first_lane(hit));
    }
    return ~0u;
}

// Write the k-mers of a labelling batch into the bitmaps and the table.
__device__ __forceinline__ void cl_write_batch(const Ctx &c, uint32_t tl, uint32_t B)
{
    const uint32_t L = c.L, k = c.k, lane = lane_id();
    for (uint32_t i = 0; i < B; ++i) {
        const uint32_t a = uniform(lds_peek(&c.banc[i]));
        const uint32_t om = a >> 31, site = a & 0x7FFFFFFFu;
        const uint32_t ay = fdiv(site, c.fL), ax = site - ay * L;
        if (om == 0) {
            set_run_plain(c, c.ohr, ay, ax, k);   // along its row
            for (uint32_t j = lane; j < k; j += 64) {   // across its columns
                uint32_t col = ax + j;
                col = col >= L ? col - L : col;
                or_l2(&c.ohc[word_tiled(c, col, ay >> 6)], 1ull << (ay & 63u));
            }
            if (lane == 0) or_l2(&c.ahr[word_plain(c, ay, ax >> 6)], 1ull << (ax & 63u));
        } else {
            set_run_plain(c, c.ovc, ax, ay, k);   // along its column
            for (uint32_t j = lane; j < k; j += 64) {   // across its rows
                uint32_t row = ay + j;
                row = row >= L ? row - L : row;
                or_l2(&c.ovr[word_tiled(c, row, ax >> 6)], 1ull << (ax & 63u));
            }
            if (lane == 0) or_l2(&c.avc[word_plain(c, ax, ay >> 6)], 1ull << (ay & 63u));
        }
        if (lane == 0) kh_insert(c, om * L * L + site, tl + i);
    }
}

// Contact f of deposit m (anchor ay, ax, orientation om) on the compressed
// lattice: whether a neighbouring k-mer's contact starts there (the first
// contact of that k-mer on this side, the side's first contact, or an end),
// and that k-mer's canonical placement index.  `back` is the anchor found
// before the side's first site (only read at f == side start with an H
// (resp. V) k-mer along the side that is not anchored there).
struct ClContact {
    bool emit;
    uint32_t P;
};

// A placement index no k-mer has (its table key would be 0xFFFFFFFF): a
// lookup of it fails and the broken invariant is reported.
constexpr uint32_t kNoPlacement = 0xFFFFFFFEu;

__device__ __forceinline__ ClContact cl_contact(const Ctx &c, uint32_t om, uint32_t ay, uint32_t ax, uint32_t f,
                                                uint32_t back0, uint32_t back1)
{
    const uint32_t L = c.L, k = c.k;
    ClContact r;
    r.emit = false;
    r.P = 0;
    const uint32_t L2 = L * L;
    const auto wrap = [&](uint32_t v) { return v >= L ? v - L : v; };
    if (f < 2 * k) {
        const uint32_t side = f < k ? 0u : 1u, j = f - side * k;
        if (om == 0) {   // rows ay -+ 1, columns ax + j
            const uint32_t row = side ? wrap(ay + 1) : wrap(ay + L - 1), col = wrap(ax + j);
            if (bit_tiled(c, c.ovr, row, col)) {
                // a V k-mer crossing the row ends at ay - 1 / starts at ay + 1
                const uint32_t ar = side ? wrap(ay + 1) : wrap(ay + L - k);
                r.emit = true;
                r.P = L2 + ar * L + col;
            } else if (bit_plain(c, c.ohr, row, col)) {
                const bool anc = bit_plain(c, c.ahr, row, col) != 0;
                if (anc || j == 0) {
                    const uint32_t ac = anc ? col : (side ? back1 : back0);
                    r.emit = true;
                    r.P = ac != ~0u ? row * L + ac : kNoPlacement;
                }
            }
        } else {         // columns ax -+ 1, rows ay + j
            const uint32_t col = side ? wrap(ax + 1) : wrap(ax + L - 1), row = wrap(ay + j);
            if (bit_tiled(c, c.ohc, col, row)) {
                // an H k-mer crossing the column ends at ax - 1 / starts at ax + 1
                const uint32_t ac = side ? wrap(ax + 1) : wrap(ax + L - k);
                r.emit = true;
                r.P = row * L + ac;
            } else if (bit_plain(c, c.ovc, col, row)) {
                const bool anc = bit_plain(c, c.avc, col, row) != 0;
                if (anc || j == 0) {
                    const uint32_t ar = anc ? row : (side ? back1 : back0);
                    r.emit = true;
                    r.P = ar != ~0u ? L2 + ar * L + col : kNoPlacement;
                }
            }
        }
    }
    return r;
}

// Census of the jammed state on the compressed lattice (Eq. 12): over every
// site and its right (lower) neighbour, pairs of occupied sites in different
// k-mers, both H, both V or perpendicular.  Two H sites side by side along a
// row are different k-mers exactly when the right one is an anchor (and
// k < L); two V sites side by side along a row always are.  Likewise down
// the columns.
template <uint32_t NT>
__device__ __forceinline__ void contact_census_bits(const Ctx &c, uint32_t tid)
{
    const uint32_t L = c.L, nw = c.nlw;
    const uint32_t tail = L & 63u;
    const bool kfull = c.k == L;
    uint64_t n[3] = {0, 0, 0};
    // dir 0: rows (H along, V across); dir 1: columns (V along, H across)
    for (uint32_t dir = 0; dir < 2; ++dir) {
        const uint64_t *along = dir ? c.ovc : c.ohr;   // same orientation as the line
        const uint64_t *anc = dir ? c.avc : c.ahr;
        const uint64_t *cross = dir ? c.ohc : c.ovr;   // the other orientation, tiled
        for (uint32_t i = tid; i < L * nw; i += NT) {
            const uint32_t line = i / nw, w = i - line * nw;
            const uint32_t wn = w + 1 == nw ? 0u : w + 1;   // next word (round the seam)
            const uint32_t valid = w + 1 == nw && tail ? tail : 64u;
            const uint64_t vmask = valid == 64 ? ~0ull : ((1ull << valid) - 1);
            const uint64_t s = ld_l2(&along[word_plain(c, line, w)]);
            const uint64_t x = ld_l2(&cross[word_tiled(c, line, w)]);
            const uint64_t a = ld_l2(&anc[word_plain(c, line, w)]);
            const uint64_t s1 = ld_l2(&along[word_plain(c, line, wn)]) & 1ull;
            const uint64_t x1 = ld_l2(&cross[word_tiled(c, line, wn)]) & 1ull;
            const uint64_t a1 = ld_l2(&anc[word_plain(c, line, wn)]) & 1ull;
            // the neighbour one step along the line, bit for bit
            const uint64_t sn = (s >> 1) | (s1 << (valid - 1));
            const uint64_t xn = (x >> 1) | (x1 << (valid - 1));
            const uint64_t an = (a >> 1) | (a1 << (valid - 1));
            const uint64_t same_o = kfull ? 0ull : (s & sn & an);   // along-orientation pair, new k-mer
            const uint64_t cross_o = x & xn;                        // across-orientation pair
            const uint64_t perp = (s & xn) | (x & sn);
            // dir 0: along = H -> n_x, across = V -> n_y; dir 1 the opposite
            n[dir] += (uint64_t)__popcll(same_o & vmask);
            n[1 - dir] += (uint64_t)__popcll(cross_o & vmask);
            n[2] += (uint64_t)__popcll(perp & vmask);
        }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint64_t w = wave_sum64(n[j]);
        if ((tid & 63) == 0 && w) atomicAdd(&c.h->ncon[j], (unsigned long long)w);
    }
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
            ax += c.s_dx()[x];
            ay += c.s_dy()[x];
            x = p;
            break;
        }
        int32_t hx = c.s_dx()[x] + c.s_dx()[p], hy = c.s_dy()[x] + c.s_dy()[p];
        c.s_par[x] = gp;
        c.s_dx()[x] = hx;
        c.s_dy()[x] = hy;
        ax += hx;
        ay += hy;
        x = gp;
    }
    dx = ax;
    dy = ay;
    return x;
}

// Contact q of a batch starting at deposit tl: deposit m = tl + q / (2k+2),
// index ci of the contact along it, the site ii of m it touches, the unit
// step e and the neighbouring site b = anchor_m + ii * u_m + e (mod L).
struct Contact {
    bool act;
    uint32_t m, ci, bx, by;
    int32_t ii, ex, ey, umx, umy;
};

__device__ __forceinline__ Contact contact_of(const Ctx &c, uint32_t tl, uint32_t q, uint32_t total)
{
    const uint32_t L = c.L, k = c.k;
    Contact ct;
    ct.act = q < total;
    const uint32_t i = ct.act ? fdiv(q, c.fC) : 0;
    ct.ci = q - i * (2 * k + 2);
    ct.m = tl + i;
    const uint32_t am = c.banc[i];
    const uint32_t om = am >> 31, site = am & 0x7FFFFFFFu;
    const uint32_t ay = fdiv(site, c.fL), ax = site - ay * L;
    ct.umx = om ? 0 : 1;
    ct.umy = om ? 1 : 0;
    if (ct.ci < k) {
        ct.ii = (int32_t)ct.ci;
        ct.ex = om ? -1 : 0;
        ct.ey = om ? 0 : -1;
    } else if (ct.ci < 2 * k) {
        ct.ii = (int32_t)(ct.ci - k);
        ct.ex = om ? 1 : 0;
        ct.ey = om ? 0 : 1;
    } else if (ct.ci == 2 * k) {
        ct.ii = 0;
        ct.ex = -ct.umx;
        ct.ey = -ct.umy;
    } else {
        ct.ii = (int32_t)k - 1;
        ct.ex = ct.umx;
        ct.ey = ct.umy;
    }
    int32_t bx = (int32_t)ax + ct.ii * ct.umx + ct.ex, by = (int32_t)ay + ct.ii * ct.umy + ct.ey;
    bx = bx >= (int32_t)L ? bx - (int32_t)L : (bx < 0 ? bx + (int32_t)L : bx);
    by = by >= (int32_t)L ? by - (int32_t)L : (by < 0 ? by + (int32_t)L : by);
    ct.bx = (uint32_t)bx;
    ct.by = (uint32_t)by;
    return ct;
}

struct LabelState {
    uint32_t base;   // k-mers base .. base+nb-1 own slots 0 .. nb-1
    uint32_t nb;
    uint32_t tl;     // first deposit of the batch (anchors in banc[n - tl])
    int32_t nx, ny;
};

__device__ __forceinline__ void reset_slots(const Ctx &c, const LabelState &ls)
{
    const uint32_t lane = lane_id();
    for (uint32_t s = lane; s < ls.nb; s += 64) {
        c.s_par[s] = s;
        c.s_dx()[s] = 0;
        c.s_dy()[s] = 0;
        c.s_meta()[s] = 0;
        c.s_gid()[s] = ls.base + s;
    }
    for (uint32_t i = lane; i < kHash; i += 64) c.h_key[i] = 0;
    if (lane == 0) c.h->nslots = ls.nb;
}

// Write the local forest back into the global one.
__device__ __forceinline__ void write_back(const Ctx &c)
{
    const uint32_t lane = lane_id();
    const uint32_t ns = c.h->nslots;
    for (uint32_t s = lane; s < ns; s += 64) {
        uint32_t x = s;
        int32_t dx = 0, dy = 0;
        for (uint32_t it = 0; it < kSlots && c.s_par[x] != x; ++it) {
            dx += c.s_dx()[x];
            dy += c.s_dy()[x];
            x = c.s_par[x];
        }
        uint32_t g = c.s_gid()[s];
        if (x == s)
            c.node[g] = make_int4((int)g, 0, 0, (int)c.s_meta()[s]);
        else
            c.node[g] = make_int4((int)c.s_gid()[x], dx, dy, 0);
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
        c.s_dx()[s] = 0;
        c.s_dy()[s] = 0;
        c.s_meta()[s] = meta;
        c.s_gid()[s] = root;
        c.h_val()[pos] = s;
    }
    __builtin_amdgcn_wave_barrier();
    uint32_t slot = 0;
    if (local) slot = id - ls.base;
    if (global) slot = c.h_val()[pos];
    return slot;
}

// Resolve the chunk's edges to slots, then merge in deposit order.
__device__ __forceinline__ void process_chunk(const Ctx &c, LabelState &ls, uint32_t ne)
{
    const uint32_t lane = lane_id();
    if (ne == 0) return;
    const bool prof = c.prof != nullptr;
    uint64_t p0 = prof ? tick() : 0;
    // every edge can bring two new roots; make room first
    if (c.h->nslots + 2 * ne > kSlots) {
        prof_add(c, kProfLabFlushes, 1);
        write_back(c);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        uint32_t m_first = c.e_step[0];
        uint32_t end = ls.base + ls.nb;
        ls.base = m_first + 1;
        ls.nb = end - ls.base;
        reset_slots(c, ls);
        __builtin_amdgcn_wave_barrier();
    }
    const uint32_t L = c.L, nC = 2 * c.k + 2;
    for (uint32_t e0 = 0; e0 < ne; e0 += 64) {
        uint32_t e = e0 + lane;
        bool act = e < ne;
        uint32_t m = act ? c.e_step[e] : 0;
        uint32_t n = act ? c.e_ms()[e] : 0;
        // the neighbour's anchor (read now, used after the finds)
        uint32_t an = 0;
        if (act) an = n >= ls.tl ? c.banc[n - ls.tl] : c.kmer[n];
        int32_t dmx, dmy, dnx, dny;
        uint32_t sm = resolve_slot(c, ls, act, m, dmx, dmy);
        uint32_t sn = resolve_slot(c, ls, act, n, dnx, dny);
        if (act) {
            // v = anchor_m - anchor_n through this contact, unwrapped
            const Contact ct = contact_of(c, ls.tl, (m - ls.tl) * nC + (uint32_t)c.e_vx()[e], 0xFFFFFFFFu);
            const uint32_t on = an >> 31, ns = an & 0x7FFFFFFFu;
            const uint32_t ny_ = fdiv(ns, c.fL), nx_ = ns - ny_ * L;
            int32_t j = on ? (int32_t)ct.by - (int32_t)ny_ : (int32_t)ct.bx - (int32_t)nx_;
            j = j < 0 ? j + (int32_t)L : j;
            const int32_t unx = on ? 0 : 1, uny = on ? 1 : 0;
            const int32_t vx = j * unx - ct.ii * ct.umx - ct.ex;
            const int32_t vy = j * uny - ct.ii * ct.umy - ct.ey;
            c.e_ms()[e] = sm | (sn << 16);
            c.e_vx()[e] = vx + dnx - dmx;
            c.e_vy()[e] = vy + dny - dmy;
        }
    }
    __builtin_amdgcn_wave_barrier();
    if (prof) {
        uint64_t p1 = tick();
        prof_add(c, kProfLabResolve, p1 - p0);
        p0 = p1;
    }
    // merge in deposit order (every lane walks the same list)
    int32_t nx = ls.nx, ny = ls.ny;
    for (uint32_t e = 0; e < ne; ++e) {
        uint32_t ms = c.e_ms()[e];
        int32_t vx = c.e_vx()[e], vy = c.e_vy()[e];
        int32_t dax, day, dbx, dby;
        uint32_t ra = local_find(c, ms & 0xFFFFu, dax, day);
        uint32_t rb = local_find(c, ms >> 16, dbx, dby);
        if (ra != rb) {
            uint32_t ma = c.s_meta()[ra], mb = c.s_meta()[rb];
            if ((ma & 0xFFu) < (mb & 0xFFu)) {
                c.s_par[ra] = rb;
                c.s_dx()[ra] = vx - dax + dbx;
                c.s_dy()[ra] = vy - day + dby;
                c.s_meta()[rb] = mb | (ma & 0x300u);
            } else {
                c.s_par[rb] = ra;
                c.s_dx()[rb] = dax - dbx - vx;
                c.s_dy()[rb] = day - dby - vy;
                uint32_t bump = (ma & 0xFFu) == (mb & 0xFFu) ? 1u : 0u;
                c.s_meta()[ra] = (ma | (mb & 0x300u)) + bump;
            }
        } else {
            int32_t wx = dax - dbx - vx, wy = day - dby - vy;
            if (wx != 0 || wy != 0) {
                uint32_t step = c.e_step[e];
                c.s_meta()[ra] |= (wx != 0 ? 0x100u : 0u) | (wy != 0 ? 0x200u : 0u);
                if (wx != 0 && nx < 0) nx = (int32_t)step + 1;
                if (wy != 0 && ny < 0) ny = (int32_t)step + 1;
            }
        }
    }
    ls.nx = nx;
    ls.ny = ny;
    __builtin_amdgcn_wave_barrier();
    if (prof) prof_add(c, kProfLabMerge, tick() - p0);
}

// fill_map: a fresh sample's site map is still to be set to -1 (empty).
// This wave does it before it reads or writes any site; the selecting
// waves never touch the map, so they start without waiting for it.
template <int G, bool SIDE>
__device__ __forceinline__ void labeler(Ctx &c, bool track, bool fill_map)
{
    const uint32_t lane = lane_id();
    const uint32_t L = c.L, k = c.k, nC = 2 * k + 2;
    const bool cl = SIDE && c.compressed;
    if (fill_map && cl) {
        // the compressed lattice: six bitmaps and the placement table, zero
        // (each bitmap area is a whole number of 128-byte tiles)
        const size_t nwb = (size_t)c.nlw * c.nt16 * 16;
        uint64_t *const bms[6] = {c.ohr, c.ovr, c.ohc, c.ovc, c.ahr, c.avc};
        for (int b = 0; b < 6; ++b) {
            ulonglong2 *q = (ulonglong2 *)bms[b];
            for (size_t i = lane; i < nwb / 2; i += 64) q[i] = make_ulonglong2(0ull, 0ull);
        }
        ulonglong2 *hq = (ulonglong2 *)c.khash;
        for (size_t i = lane; i < ((size_t)1 << c.hlg) / 2; i += 64) hq[i] = make_ulonglong2(0ull, 0ull);
        __builtin_amdgcn_s_waitcnt(0);   // the zeros are in L2 before any atomic on them
    } else if (fill_map) {
        // the padded map (a multiple of 32 x 32 sites)
        int4 *m4 = (int4 *)c.map;
        const size_t q4 = (size_t)c.lp() * c.lp() / 4;
        for (size_t i = lane; i < q4; i += 64) m4[i] = make_int4(-1, -1, -1, -1);
    }
    const FastDiv fC = c.fC;
    LabelState ls;
    ls.nx = c.h->nx;
    ls.ny = c.h->ny;
    uint32_t tl = c.h->t0;
    const bool prof = c.prof != nullptr;
    uint64_t p_start = prof ? tick() : 0, p0 = 0;
    uint64_t p_idle = 0, p_map = 0, p_gather = 0, p_batches = 0, p_edges = 0;
    // a run that resumes after labelling ended early has nothing to label
    bool stopped = c.h->lab_stop != 0;
    while (!stopped) {
        uint32_t sp;
        bool finished = false;
        if (prof) p0 = tick();
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
        if (prof) {
            uint64_t p1 = tick();
            p_idle += p1 - p0;
            p0 = p1;
            ++p_batches;
        }
        if (finished) break;
        const uint32_t B = sp - tl < kBatch ? sp - tl : kBatch;
        const uint32_t t1 = tl + B;
        // take the placements out of the ring
        if (lane < B) {
            uint32_t P = c.ring[(tl + lane) & (kRing - 1)];
            uint32_t o = P >= c.L2() ? 1u : 0u;
            uint32_t a = (P - o * c.L2()) | (o << 31);
            c.banc[lane] = a;
            c.kmer[tl + lane] = a;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) lds_store(&c.h->lab_progress, t1);
        // site map of the batch; long k-mers (sparse-clear kernels) walk
        // each k-mer along its line, decoding its anchor once
        if (cl) {
            cl_write_batch(c, tl, B);
            __builtin_amdgcn_s_waitcnt(0);   // every atomic of the batch done before its reads
        } else if (SIDE && k >= kSideGather) {
            for (uint32_t i = 0; i < B; ++i) {
                const uint32_t a = uniform(lds_peek(&c.banc[i]));
                const uint32_t om = a >> 31, site = a & 0x7FFFFFFFu;
                const uint32_t ay = fdiv(site, c.fL), ax = site - ay * L;
                const uint32_t along0 = om ? ay : ax;
                for (uint32_t j = lane; j < k; j += 64) {
                    uint32_t al = along0 + j;
                    al = al >= L ? al - L : al;
                    c.map[om ? map_index(c, al, ax) : map_index(c, ay, al)] = (int32_t)(tl + i);
                }
            }
        }
        for (uint32_t q = lane; !cl && !(SIDE && k >= kSideGather) && q < B * k; q += 64) {
            uint32_t i = fdiv(q, c.fk);
            uint32_t s = q - i * k;
            uint32_t a = c.banc[i];
            uint32_t site = a & 0x7FFFFFFFu;
            uint32_t ay = fdiv(site, c.fL), ax = site - ay * L;
            if (a >> 31) {
                ay += s;
                ay = ay >= L ? ay - L : ay;
            } else {
                ax += s;
                ax = ax >= L ? ax - L : ax;
            }
            c.map[map_index(c, ay, ax)] = (int32_t)(tl + i);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        if (prof) {
            uint64_t p1 = tick();
            p_map += p1 - p0;
            p0 = p1;
        }
        ls.base = tl;
        ls.nb = B;
        ls.tl = tl;
        reset_slots(c, ls);
        __builtin_amdgcn_wave_barrier();
        // contacts of every deposit of the batch, in deposit order:
        // c in [0,k): above (H) / left (V) of site c; [k,2k): below / right;
        // 2k: before site 0; 2k+1: after site k-1.  G rounds of 64 contacts
        // have their map reads in flight together.  A contact with the same
        // neighbour as the previous one on the same side has the same vector
        // v (their offsets along both k-mers move together) unless k = L,
        // where a run can pass the seam; such repeats are dropped.  The
        // edge keeps the contact index; v is formed once the neighbour's
        // anchor has been read, next to the cluster finds.
        uint32_t ne = 0;
        int32_t cn = -1;
        const uint32_t total = B * nC;
        const bool dedupe = k != L;
        bool stop = false;
        const bool side_gather = SIDE && k >= kSideGather;
        if (cl) {
            // compressed lattice: the sides are read a word (64 sites) per
            // lane; a neighbour k-mer's contact starts where its anchor or its
            // crossing is met (or at the side's first site); the candidates
            // go through the placement table together
            for (uint32_t i = 0; i < B && !stop; ++i) {
                const uint32_t m = tl + i;
                const uint32_t a = uniform(lds_peek(&c.banc[i]));
                const uint32_t om = a >> 31, site = a & 0x7FFFFFFFu;
                const uint32_t ay = fdiv(site, c.fL), ax = site - ay * L;
                const auto wrap = [&](uint32_t v) { return v >= L ? v - L : v; };
                // sides: H deposit rows ay -+ 1 along columns from ax (H occupancy
                // along, V across); V deposit columns ax -+ 1 along rows from ay
                const uint64_t *const along = om ? c.ovc : c.ohr;
                const uint64_t *const cross = om ? c.ohc : c.ovr;
                const uint64_t *const anc = om ? c.avc : c.ahr;
                const uint32_t pst = om ? ay : ax;
                const uint32_t line0 = om ? wrap(ax + L - 1) : wrap(ay + L - 1);
                const uint32_t line1 = om ? wrap(ax + 1) : wrap(ay + 1);
                const Span sp = make_span(c, pst, k);
                // ---- reads: the first site of each side, the end sites, the words
                const uint32_t f0a = bit_plain(c, along, line0, pst), f0n = bit_plain(c, anc, line0, pst);
                const uint32_t f1a = bit_plain(c, along, line1, pst), f1n = bit_plain(c, anc, line1, pst);
                // ends (before site 0, after site k-1): occupied along the deposit's
                // own line (same orientation) or across it
                const uint32_t e0 = om ? wrap(ay + L - 1) : wrap(ax + L - 1);
                const uint32_t e1 = om ? wrap(ay + k) : wrap(ax + k);
                const uint32_t own = om ? ax : ay;   // the deposit's own line
                const uint32_t e0s = bit_plain(c, along, own, e0), e1s = bit_plain(c, along, own, e1);
                const uint32_t e0x = bit_tiled(c, cross, own, e0), e1x = bit_tiled(c, cross, own, e1);
                // ---- anchors found by search (only where needed)
                const uint32_t back0 = (f0a && !f0n) ? nearest_before(c, anc, line0, pst, k - 1) : ~0u;
                const uint32_t back1 = (f1a && !f1n) ? nearest_before(c, anc, line1, pst, k - 1) : ~0u;
                // a k-mer across the deposit's line at an end: its anchor is the
                // nearest one before along the end's line (the other bitmap)
                const uint64_t *const anc_x = om ? c.ahr : c.avc;
                const uint32_t x0 = (!e0s && e0x) ? nearest_before(c, anc_x, e0, own, k - 1) : ~0u;
                const uint32_t x1 = (!e1s && e1x) ? nearest_before(c, anc_x, e1, own, k - 1) : ~0u;
                // ---- candidates, 64 per round: lane l takes word item l of the
                // two sides' windows (first round), then the ends
                const uint32_t nitems = 2 * sp.n;
                for (uint32_t r0 = 0; r0 < nitems + 2 && !stop; r0 += 64) {
                    const uint32_t it = r0 + lane;
                    uint64_t emitA = 0, emitX = 0;   // along / across contacts in this lane's word
                    uint32_t sd = 0, w = 0;
                    if (it < nitems) {
                        sd = it >= sp.n ? 1u : 0u;
                        w = span_block(sp, it - sd * sp.n);
                        const uint32_t ln = sd ? line1 : line0;
                        const uint64_t wa = ld_l2(&along[word_plain(c, ln, w)]);
                        const uint64_t wx = ld_l2(&cross[word_tiled(c, ln, w)]);
                        const uint64_t wn = ld_l2(&anc[word_plain(c, ln, w)]);
                        // window positions in this word: [pst, pst + k) cyclic
                        const uint32_t b0 = w * 64;
                        uint64_t win = 0;
                        {
                            const uint32_t e1p = pst + k < L ? pst + k : L;   // [pst, e1p)
                            const int32_t lo = (int32_t)(pst > b0 ? pst : b0), hi = (int32_t)(e1p < b0 + 64 ? e1p : b0 + 64);
                            if (lo < hi) win |= bit_range(lo - (int32_t)b0, hi - 1 - (int32_t)b0);
                            if (pst + k > L) {   // [0, pst + k - L)
                                const uint32_t e2p = pst + k - L;
                                const int32_t hi2 = (int32_t)(e2p < b0 + 64 ? e2p : b0 + 64);
                                if ((int32_t)b0 < hi2) win |= bit_range(0, hi2 - 1 - (int32_t)b0);
                            }
                        }
                        const uint64_t first = (pst >> 6) == w ? (1ull << (pst & 63u)) : 0ull;
                        emitX = wx & win;
                        emitA = wa & win & (wn | first);
                    } else if (it < nitems + 2) {
                        // ends: one contact each, carried in bit 0
                        const uint32_t e = it - nitems;
                        const uint32_t es = e ? e1s : e0s, ex = e ? e1x : e0x;
                        emitA = es ? 1ull : 0ull;
                        emitX = (!es && ex) ? 1ull : 0ull;
                        sd = 2 + e;
                    }
                    // one candidate per lane per pass until every lane is done
                    for (;;) {
                        const bool have = (emitA | emitX) != 0;
                        if (__ballot(have) == 0) break;
                        uint32_t f = 0, P = kNoPlacement;
                        if (have) {
                            const bool isA = emitA != 0;
                            const uint64_t bits = isA ? emitA : emitX;
                            const uint32_t b = (uint32_t)(__ffsll((long long)bits) - 1);
                            if (isA) emitA &= emitA - 1; else emitX &= emitX - 1;
                            if (sd < 2) {
                                const uint32_t pos = w * 64 + b;               // along the side line
                                uint32_t j = pos + L - pst;
                                j = j >= L ? j - L : j;
                                f = sd * k + j;
                                const uint32_t ln = sd ? line1 : line0;
                                if (isA) {
                                    // a k-mer along the side: anchored here, or (first site)
                                    // at the anchor found before it
                                    const uint32_t an = (pos == pst && !(sd ? f1n : f0n)) ? (sd ? back1 : back0) : pos;
                                    if (an != ~0u) P = om ? (L * L + an * L + ln) : (ln * L + an);
                                } else {
                                    // a k-mer across the side ends (side 0) or starts (side 1)
                                    // next to the deposit's line
                                    const uint32_t at = sd ? (own + 1 == L ? 0u : own + 1) : wrap(own + L - k);
                                    P = om ? (pos * L + at) : (L * L + at * L + pos);
                                }
                            } else {
                                const uint32_t e = sd - 2;
                                f = 2 * k + e;
                                const uint32_t ep = e ? e1 : e0;   // position of the end on the own line
                                if (isA) {
                                    // a k-mer along the deposit's line ends at / starts after it
                                    const uint32_t at = e ? ep : wrap(pst + L - (k % L));
                                    P = om ? (L * L + at * L + own) : (own * L + at);
                                } else {
                                    const uint32_t an = e ? x1 : x0;   // anchor on the end's line
                                    if (an != ~0u) P = om ? (ep * L + an) : (L * L + an * L + ep);
                                }
                            }
                        }
                        int32_t n = -1;
                        if (have) n = kh_find(c, P);
                        if (have && n < 0) c.h->status = kErrLabel;   // an occupied site with no k-mer
                        const bool keep = n >= 0 && (uint32_t)n <= m;
                        const uint64_t bal = __ballot(keep);
                        if (keep) {
                            const uint32_t idx = ne + lanes_below(bal);
                            c.e_step[idx] = m;
                            c.e_ms()[idx] = (uint32_t)n;
                            c.e_vx()[idx] = (int32_t)f;
                        }
                        ne += (uint32_t)__popcll(bal);
                        __builtin_amdgcn_wave_barrier();
                        if (ne + 64 > kEdges) {
                            if (prof) {
                                p_gather += tick() - p0;
                                p_edges += ne;
                            }
                            process_chunk(c, ls, ne);
                            if (prof) p0 = tick();
                            ne = 0;
                            if (!track && ls.nx >= 0 && ls.ny >= 0) stop = true;
                            if (c.h->status != 0) stop = true;
                            if (stop) break;
                        }
                    }
                }
                if (i + 1 == B && !stop) {
                    if (prof) {
                        p_gather += tick() - p0;
                        p_edges += ne;
                    }
                    process_chunk(c, ls, ne);
                    if (prof) p0 = tick();
                    ne = 0;
                    if (!track && ls.nx >= 0 && ls.ny >= 0) stop = true;
                    if (c.h->status != 0) stop = true;
                }
            }
        } else if (side_gather) {
            // Long k-mers: deposit by deposit, side by side.  A side's
            // contacts lie on one lattice line (the row above / below an H
            // k-mer, the column left / right of a V one), so lane j's site
            // is j steps along it; the two ends follow as a short third side.
            // Fewer instructions per contact, but one flight of reads per
            // side: it pays once a side is several flights long.
            for (uint32_t i = 0; i < B && !stop; ++i) {
                const uint32_t m = tl + i;
                const uint32_t a = uniform(lds_peek(&c.banc[i]));
                const uint32_t om = a >> 31, site = a & 0x7FFFFFFFu;
                const uint32_t ay = fdiv(site, c.fL), ax = site - ay * L;
                const uint32_t along0 = om ? ay : ax;   // coordinate along the k-mer
                const uint32_t across = om ? ax : ay;   // the other one
                for (uint32_t side = 0; side < 3 && !stop; ++side) {
                    const uint32_t len = side < 2 ? k : 2u;
                    const uint32_t fix = side == 0 ? (across == 0 ? L - 1 : across - 1)
                                                   : (across + 1 == L ? 0u : across + 1);
                    cn = -1;
                    for (uint32_t j0 = 0; j0 < len && !stop; j0 += 64 * G) {
                        int32_t nval[G];
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            const uint32_t j = j0 + 64 * g + lane;
                            int32_t v = -1;
                            if (j < len) {
                                // sides: along0 + j; ends: one before site 0, one after site k-1
                                uint32_t al = side < 2 ? along0 + j : (j == 0 ? along0 + L - 1 : along0 + k);
                                al = al >= L ? al - L : al;
                                const uint32_t cr = side < 2 ? fix : across;
                                v = c.map[om ? map_index(c, al, cr) : map_index(c, cr, al)];
                            }
                            nval[g] = v;
                        }
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            const uint32_t jr = j0 + 64 * g;
                            if (jr >= len || stop) continue;
                            const uint32_t j = jr + lane;
                            const int32_t n = nval[g];
                            const bool keep = j < len && n >= 0 && (uint32_t)n <= m;
                            const int32_t key = keep ? n : -1;
                            const int32_t pn = from_previous_lane(key, cn);
                            const bool emit = keep && !(dedupe && side < 2 && j > 0 && pn == n);
                            cn = (int32_t)bcast((uint32_t)key, 63);
                            const uint64_t bal = __ballot(emit);
                            if (emit) {
                                const uint32_t idx = ne + lanes_below(bal);
                                c.e_step[idx] = m;
                                c.e_ms()[idx] = (uint32_t)n;
                                c.e_vx()[idx] = (int32_t)(side < 2 ? side * k + j : 2 * k + j);
                            }
                            ne += (uint32_t)__popcll(bal);
                            __builtin_amdgcn_wave_barrier();
                            const bool last = i + 1 == B && side == 2 && jr + 64 >= len;
                            if (ne + 64 > kEdges || last) {
                                if (prof) {
                                    p_gather += tick() - p0;
                                    p_edges += ne;
                                }
                                process_chunk(c, ls, ne);
                                if (prof) p0 = tick();
                                ne = 0;
                                if (!track && ls.nx >= 0 && ls.ny >= 0) stop = true;
                                if (c.h->status != 0) stop = true;
                            }
                        }
                    }
                }
            }
        }
        for (uint32_t g0 = 0; !cl && !side_gather && g0 < total && !stop; g0 += 64 * G) {
            int32_t nval[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                Contact ct = contact_of(c, tl, g0 + 64 * g + lane, total);
                nval[g] = ct.act ? c.map[map_index(c, ct.by, ct.bx)] : -1;
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const uint32_t q0 = g0 + 64 * g;
                if (q0 >= total || stop) continue;
                const uint32_t q = q0 + lane;
                const bool act = q < total;
                const uint32_t i = act ? fdiv(q, fC) : 0;
                const uint32_t ci = q - i * nC;
                const uint32_t m = tl + i;
                const int32_t n = nval[g];
                const bool keep = act && n >= 0 && (uint32_t)n <= m;
                const int32_t key = keep ? n : -1;
                int32_t pn = __shfl_up(key, 1, 64);
                if (lane == 0) pn = cn;
                const bool same_run = ci > 0 && ci < 2 * k && ci != k;
                const bool emit = keep && !(dedupe && same_run && pn == n);
                cn = (int32_t)bcast((uint32_t)key, 63);
                uint64_t bal = __ballot(emit);
                uint32_t off = (uint32_t)__popcll(bal & ((1ull << lane) - 1));
                if (emit) {
                    uint32_t idx = ne + off;
                    c.e_step[idx] = m;
                    c.e_ms()[idx] = (uint32_t)n;
                    c.e_vx()[idx] = (int32_t)ci;
                }
                ne += (uint32_t)__popcll(bal);
                __builtin_amdgcn_wave_barrier();
                if (ne + 64 > kEdges || q0 + 64 >= total) {
                    if (prof) {
                        p_gather += tick() - p0;
                        p_edges += ne;
                    }
                    process_chunk(c, ls, ne);
                    if (prof) p0 = tick();
                    ne = 0;
                    if (!track && ls.nx >= 0 && ls.ny >= 0) stop = true;
                    if (c.h->status != 0) stop = true;
                }
            }
        }
        if (stop) {
            stopped = true;
            break;
        }
        if (prof) p0 = tick();
        write_back(c);
        if (prof) prof_add(c, kProfLabWriteBack, tick() - p0);
        tl = t1;
    }
    if (prof) {
        prof_add(c, kProfLabTotal, tick() - p_start);
        prof_add(c, kProfLabIdle, p_idle);
        prof_add(c, kProfLabMap, p_map);
        prof_add(c, kProfLabGather, p_gather);
        prof_add(c, kProfLabBatches, p_batches);
        prof_add(c, kProfLabEdges, p_edges);
    }
    if (lane == 0) {
        c.h->nx = ls.nx;
        c.h->ny = ls.ny;
        c.h->lab_stop = stopped ? 1u : 0u;
        lds_store(&c.h->lab_exit, 1u);
    }
}

// ---------------------------------------------------------------------------
// Contact census at jamming (Eq. 12)
// ---------------------------------------------------------------------------

// Every site and its right and lower neighbour (mod L): a pair of occupied
// sites in different k-mers counts as both horizontal, both vertical or
// perpendicular (orientation from the k-mer records).  The workgroup walks
// the map tile by tile in memory order, 32 lanes per 128-byte tile and
// kCensusUnroll tiles per lane group in flight.
constexpr uint32_t kCensusUnroll = 4;

template <uint32_t NT>
__device__ __forceinline__ void contact_census(const Ctx &c, uint32_t tid)
{
    const uint32_t L = c.L;
    const uint32_t groups = NT / 32;            // tiles per pass
    const uint32_t grp = tid >> 5, off = tid & 31;
    const uint32_t oy = off >> c.lg_mc(), ox = off & c.mc_m();
    const uint32_t ntr = c.lp() >> c.lg_mr;       // tile rows
    const uint32_t ntiles = ntr * c.mtpr();
    uint32_t n[3] = {0, 0, 0};
    for (uint32_t t0 = 0; t0 < ntiles; t0 += groups * kCensusUnroll) {
        int32_t a[kCensusUnroll], br[kCensusUnroll], bd[kCensusUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kCensusUnroll; ++u) {
            const uint32_t tile = t0 + u * groups + grp;
            a[u] = br[u] = bd[u] = -1;
            if (tile < ntiles) {
                const uint32_t tr = tile / c.mtpr(), tc = tile - tr * c.mtpr();
                const uint32_t y = (tr << c.lg_mr) + oy, x = (tc << c.lg_mc()) + ox;
                if (y < L && x < L) {
                    a[u] = c.map[((size_t)tile << 5) + off];
                    const uint32_t xr = x + 1 == L ? 0 : x + 1, yd = y + 1 == L ? 0 : y + 1;
                    br[u] = c.map[map_index(c, y, xr)];
                    bd[u] = c.map[map_index(c, yd, x)];
                }
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kCensusUnroll; ++u) {
            if (a[u] < 0) continue;
            const uint32_t oa = c.kmer[a[u]] >> 31;
            if (br[u] >= 0 && br[u] != a[u]) {
                const uint32_t ob = c.kmer[br[u]] >> 31;
                ++n[oa != ob ? 2 : oa];
            }
            if (bd[u] >= 0 && bd[u] != a[u]) {
                const uint32_t ob = c.kmer[bd[u]] >> 31;
                ++n[oa != ob ? 2 : oa];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint32_t w = wave_sum32(n[j]);
        if ((tid & 63) == 0 && w) atomicAdd(&c.h->ncon[j], (unsigned long long)w);
    }
}

// ---------------------------------------------------------------------------
// Cluster sizes (Eq. 11)
// ---------------------------------------------------------------------------

// Histogram of the cluster sizes of k-mers 0 .. nk-1 (the whole lattice after
// deposit nk): member counts per root in the k-mer record array (no longer
// needed once labelling is done), then per root the bin of its size in
// sites, 2^b <= size < 2^(b+1).  Writes kSizeBins counters to out.
template <uint32_t NT>
__device__ __forceinline__ void size_histogram(const Ctx &c, uint32_t tid, uint32_t nk,
                                               unsigned long long *out)
{
    uint32_t *members = c.kmer;
    unsigned long long *bins = (unsigned long long *)c.h_key;   // LDS, free after labelling
    for (uint32_t i = tid; i < nk; i += NT) members[i] = 0;
    if (tid < kSizeBins) bins[tid] = 0;
    __syncthreads();
    uint32_t bad = 0;
    for (uint32_t i = tid; i < nk; i += NT) {
        uint32_t root, meta;
        int32_t dx, dy;
        if (global_find(c, i, root, dx, dy, meta) && root < nk)
            atomicAdd(&members[root], 1u);
        else
            bad = 1;
    }
    __syncthreads();
    for (uint32_t i = tid; i < nk; i += NT) {
        // the counts were formed by atomics in L2: read them there too
        const uint32_t m = __hip_atomic_load(&members[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (m) {
            const uint64_t sites = (uint64_t)m * c.k;
            atomicAdd(&bins[63 - __clzll((long long)sites)], 1ull);
        }
    }
    if (bad) atomicOr(&c.h->nonwrap, 0x80000000u);   // marks a broken forest
    __syncthreads();
    if (tid < kSizeBins) out[tid] = (c.h->nonwrap & 0x80000000u) ? ~0ull : bins[tid];
}

// ---------------------------------------------------------------------------
// One sample, then the persistent loop
// ---------------------------------------------------------------------------

__device__ __forceinline__ void carve(Ctx &c, const DevDesc &d, uint8_t *slab, uint8_t *lds)
{
    c.L = d.L;
    c.k = d.k;
    c.wd = d.wd;
    c.flags = d.flags;
    c.sample = d.sample;
    c.ncap = d.L * d.L / d.k + 1;
    c.k0 = (uint32_t)d.seed;
    c.k1 = (uint32_t)(d.seed >> 32);
    c.fL = d.fL;
    c.fk = d.fk;
    c.fC = d.fC;
    c.fwd = d.fwd;
    c.fwp = d.fwp;
    c.lg_tr = d.lg_tr;
    c.lg_mr = d.lg_mr;
    c.spec_rows = d.spec_rows;
    SlabLayout s = slab_layout(d.L, d.k, d.compressed != 0);
    c.av0 = (uint64_t *)(slab + s.avail0);
    c.av1 = (uint64_t *)(slab + s.avail1);
    c.sm0 = (uint64_t *)(slab + s.sum0);
    c.sm1 = (uint64_t *)(slab + s.sum1);
    c.map = (int32_t *)(slab + s.map);
    c.node = (int4 *)(slab + s.node);
    c.kmer = (uint32_t *)(slab + s.kmer);
    LdsLayout l = lds_layout(d.L);
    c.h = (Hdr *)(lds + l.hdr);
    c.cnt0 = (uint32_t *)(lds + l.cnt0);
    c.cnt1 = (uint32_t *)(lds + l.cnt1);
    c.cnt2 = (uint32_t *)(lds + l.cnt2);
    c.ring = (uint32_t *)(lds + l.ring);
    c.banc = (uint32_t *)(lds + l.banc);
    c.e_step = (uint32_t *)(lds + l.edges);
    c.s_par = (uint32_t *)(lds + l.slots);
    c.h_key = (uint32_t *)(lds + l.hash);
    c.interval = d.interval;
    c.hb = (uint32_t *)(slab + s.hb);
    c.vb = (uint32_t *)(slab + s.vb);
    c.ivg = d.ivg;
    c.ivstride = d.ivg ? interval_diff_words(d.k) + 68 : 0u;
    c.dD = d.ivg ? (uint32_t *)(slab + s.ivd) : (uint32_t *)(lds + l.total);
    c.dC = c.dD + interval_diff_words(d.k);
    c.fB = d.fB;
    c.compressed = d.compressed;
    c.nlw = line_words(d.L);
    c.nt16 = tile16(d.L);
    c.hlg = 31 - __clz(hash_slots(d.L, d.k));
    c.ohr = (uint64_t *)(slab + s.ohr);
    c.ovr = (uint64_t *)(slab + s.ovr);
    c.ohc = (uint64_t *)(slab + s.ohc);
    c.ovc = (uint64_t *)(slab + s.ovc);
    c.ahr = (uint64_t *)(slab + s.ahr);
    c.avc = (uint64_t *)(slab + s.avc);
    c.khash = (unsigned long long *)(slab + s.khash);
}

// One sample on one workgroup.  deadline = 0 runs it from the empty lattice
// to jamming (batched runs, slab owned by the workgroup).  Otherwise the
// slab is the sample's own and holds a SampleState: a finished sample
// re-emits its result, a yielded one restores its row counts and header and
// continues, and the run yields again at the deadline, saving them back.
template <int NSEL, int ROWW, bool SPARSE, bool CENSUS>
__device__ __forceinline__ void run_sample(const KernelArgs &a, const DevDesc &d, uint8_t *lds,
                                           uint64_t deadline)
{
    constexpr uint32_t NT = 64 * (NSEL + 1);
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid >> 6;
    uint8_t *slab = d.slab ? (uint8_t *)d.slab : a.slabs + (size_t)blockIdx.x * a.slab_stride;
    Ctx c;
    carve(c, d, slab, lds);
    c.prof = a.prof ? a.prof + (size_t)d.out * kProfSlots : nullptr;
    const uint64_t p_init = c.prof ? tick() : 0;
    const uint32_t L = c.L;
    const bool h_only = (c.flags & 1u) != 0;
    const bool track = (c.flags & 2u) != 0;
    // the contact census is compiled only into the CENSUS kernels, so that
    // the others keep their register allocation
    const bool sizes_pass = CENSUS && (d.flags & kDescSizesPass) != 0;
    const bool contacts = CENSUS && !sizes_pass && (c.flags & 4u) != 0;
    const bool sliced = deadline != 0;
    uint32_t stop = 0;
    if (sizes_pass) {
        // second pass: stop right after the first wrap the first pass found
        const int64_t nany = a.results[d.out].n_wrap_any;
        if (nany <= 0 || a.results[d.out].status != 0) {
            if (tid < kSizeBins) a.hist[(size_t)d.out * kSizeBins + tid] = nany <= 0 ? 0ull : ~0ull;
            __syncthreads();
            return;
        }
        stop = (uint32_t)nany;
    }
    SampleState *st = (SampleState *)(slab + slab_layout(d.L, d.k, d.compressed != 0).state);
    uint32_t *saved_cnt = (uint32_t *)((uint8_t *)st + kStateBytes);
    const uint32_t phase = sliced ? st->phase : 0u;
    if (phase == 2) {
        if (tid == 0) a.results[d.out] = st->result;
        __syncthreads();
        return;
    }

    if (phase == 1) {
        // ---- resume: row counts and the header from the slab
        const uint32_t nw = lds_count_bytes(L) / 4;
        for (uint32_t i = tid; i < nw; i += NT) c.cnt0[i] = saved_cnt[i];
        if (tid == 0) {
            Hdr *h = c.h;
            const uint32_t t0 = st->t;
            h->sel_progress = t0;
            h->sel_done = 0;
            h->lab_progress = t0;
            h->lab_exit = 0;
            h->clr_gen = t0;
            h->clr_done = t0 * (NSEL - 1);
            h->cur_p = 0;
            h->nslots = 0;
            h->nx = st->nx;
            h->ny = st->ny;
            h->nclusters = 0;
            h->nonwrap = 0;
            h->status = st->status;
            h->t0 = t0;
            h->p0 = st->P;
            h->wchg = st->wchg;
            h->occ = st->occ;
            h->seqh = st->seqh;
            h->resumed = 1;
            h->preempt = 0;
            h->lab_stop = st->lab_stop;
            h->stop = 0;
            h->ncon[0] = h->ncon[1] = h->ncon[2] = 0;
            for (int q = 0; q < 10; ++q) h->sel_acc[q] = 0;
        }
    } else {
        // ---- initial state (Sec. II.A): all placements free; all sites
        // empty is written by the labelling wave (fill_map below)
        // bitmaps: every anchor of a real row and column available, padding 0
        const uint32_t wd = c.wd;
        const uint32_t tailbits = L & 63u;
        const uint64_t last = tailbits ? ((1ull << tailbits) - 1) : ~0ull;
        const uint32_t nwords = c.lp() * c.wp();
        const bool iv = SPARSE && c.interval;
        for (uint32_t i = tid; i < nwords; i += NT) {
            uint32_t row = fdiv(i, c.fwp), wi = i - row * c.wp();
            uint64_t full = (row >= L || wi >= wd) ? 0ull : (wi == wd - 1 ? last : ~0ull);
            const uint32_t at = bm_index(c, row, wi);
            if (!iv) c.av0[at] = full;   // the interval clear keeps H anchors in buckets only
            c.av1[at] = h_only ? 0ull : full;
        }
        if (iv) {
            // every line one run: bucket j holds [j(k+1), min((j+1)(k+1), L) - 1]
            const uint32_t nS = num_buckets(L, c.k), B = c.k + 1;
            for (uint32_t j = 0; j < nS; ++j) {
                const uint32_t a = j * B, b = (a + B < L ? a + B : L) - 1;
                const uint32_t E = a | (b << 16);
                for (uint32_t q = tid; q < L; q += NT) {
                    c.hb[j * c.lp() + q] = E;
                    c.vb[j * c.lp() + q] = h_only ? kNoSeg : E;
                }
            }
        }
        if (SPARSE && !iv) {
            // summary bit set for every word of a real row and column
            const uint32_t nsum = c.lp() * c.swp();
            for (uint32_t i = tid; i < nsum; i += NT) {
                uint32_t row = i / c.swp(), sw = i - row * c.swp();
                uint32_t lo = sw * 64, hi = lo + 64 < wd ? lo + 64 : wd;
                uint64_t bits = (row >= L || lo >= wd) ? 0ull : (hi - lo == 64 ? ~0ull : ((1ull << (hi - lo)) - 1));
                c.sm0[i] = bits;
                c.sm1[i] = h_only ? 0ull : bits;
            }
        }
        const uint32_t rows = 2 * L;
        const uint32_t vcount = h_only ? 0u : L;
        for (uint32_t i = tid; i < (rows + 1) / 2; i += NT) {
            uint32_t r0 = 2 * i, r1 = 2 * i + 1;
            uint32_t c0 = r0 < L ? L : (r0 < rows ? vcount : 0);
            uint32_t c1 = r1 < L ? L : (r1 < rows ? vcount : 0);
            c.cnt0[i] = c0 | (c1 << 16);
        }
        for (uint32_t g = tid; g < c.n1(); g += NT) {
            uint32_t lo = g * 64, hi = lo + 64 < rows ? lo + 64 : rows;
            uint32_t nh = hi <= L ? hi - lo : (lo >= L ? 0 : L - lo);
            c.cnt1[g] = nh * L + (hi - lo - nh) * vcount;
        }
        for (uint32_t g = tid; g < c.n2(); g += NT) {
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
            h->t0 = 0;
            h->p0 = 0;
            h->wchg = 0;
            h->occ = 0;
            h->seqh = 0;
            h->resumed = 0;
            h->preempt = 0;
            h->lab_stop = 0;
            h->stop = stop;
            h->ncon[0] = h->ncon[1] = h->ncon[2] = 0;
            for (int q = 0; q < 10; ++q) h->sel_acc[q] = 0;
        }
    }
    if (SPARSE && c.interval) {
        const uint32_t n = (c.ivg ? 2u : 1u) * (interval_diff_words(c.k) + 68);
        for (uint32_t i = tid; i < n; i += NT) c.dD[i] = 0u;
        if (c.ivg) __builtin_amdgcn_s_waitcnt(0);   // slab stores done before any step's atomics
    }
    if (tid == 0) c.h->bar = 0;
    __syncthreads();
    if (c.prof && tid == 0) atomicAdd(&c.prof[kProfInit], (unsigned long long)(tick() - p_init));

    // ---- the two chains
    if (wave == 0)
        selector<NSEL, ROWW, SPARSE, CENSUS>(c, deadline);
    else if (wave < (uint32_t)NSEL)
        helper<NSEL, ROWW, SPARSE>(c, wave);
    else
        // the side-by-side gather is compiled into the sparse-clear kernels
        // only (long k-mers); it would raise the others' register count
        labeler<(NSEL >= 7 && !CENSUS ? 16 : 8), SPARSE>(c, track || contacts || sizes_pass, phase != 1);
    __syncthreads();

    if constexpr (CENSUS) {
        if (sizes_pass) {
            // ---- cluster-size histogram right after deposit `stop`; the
            // first pass's result stands
            if (c.h->status == 0 && c.h->sel_done == stop + 1) {
                size_histogram<NT>(c, tid, stop, a.hist + (size_t)d.out * kSizeBins);
            } else if (tid < kSizeBins) {
                a.hist[(size_t)d.out * kSizeBins + tid] = ~0ull;
            }
            __syncthreads();
            return;
        }
    }

    if (c.h->preempt && c.h->status == 0) {
        // ---- yield: save what the next run needs
        const uint32_t nw = lds_count_bytes(L) / 4;
        for (uint32_t i = tid; i < nw; i += NT) saved_cnt[i] = c.cnt0[i];
        if (tid == 0) {
            const Hdr *h = c.h;
            const uint32_t tdone = h->sel_done - 1;
            st->phase = 1;
            st->t = tdone;
            st->P = h->p0;
            st->lab_stop = h->lab_stop;
            st->nx = h->nx;
            st->ny = h->ny;
            st->status = 0;
            st->occ = h->occ;
            st->seqh = h->seqh;
            st->wchg = h->wchg;
            DevResult r;
            r.n_jam = tdone;   // progress so far
            r.n_wrap_x = h->nx;
            r.n_wrap_y = h->ny;
            r.n_wrap_any = -1;
            r.occ_hash = 0;
            r.seq_hash = 0;
            r.n_clusters_jam = -1;
            r.n_nonwrapping_jam = -1;
            r.status = kStatusYielded;
            r.tile = (int32_t)d.tile;
            r.alg_bytes = 0;
            r.wchg_words = h->wchg;
            r.n_contacts_x = r.n_contacts_y = r.n_contacts_xy = -1;
            a.results[d.out] = r;
        }
        __syncthreads();
        return;
    }

    // ---- contact census at jamming (Eq. 12)
    if constexpr (CENSUS) {
        if (contacts && c.h->status == 0) {
            if (SPARSE && c.compressed)
                contact_census_bits<NT>(c, tid);
            else
                contact_census<NT>(c, tid);
            __syncthreads();
        }
    }

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
        r.tile = (int32_t)d.tile;
        r.wchg_words = c.h->wchg;
        r.alg_bytes = 4 * Lw * Lw + 16 * Lw * c.wd +
                      (uint64_t)njam * (4 * kw + 4 * (2 * kw + 2) + 8 * c.wd + 16) + 16 * r.wchg_words;
        r.n_contacts_x = contacts ? (int64_t)c.h->ncon[0] : -1;
        r.n_contacts_y = contacts ? (int64_t)c.h->ncon[1] : -1;
        r.n_contacts_xy = contacts ? (int64_t)c.h->ncon[2] : -1;
        a.results[d.out] = r;
        if (sliced) {
            st->result = r;
            st->phase = 2;
        }
    }
    __syncthreads();
}

template <int NSEL, int ROWW, bool SPARSE, bool CENSUS>
__global__ __launch_bounds__(64 * (NSEL + 1)) void rsa_persistent(KernelArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t next;
    __shared__ uint64_t deadline;
    if (threadIdx.x == 0) deadline = a.quantum ? tick() + a.quantum : 0;
    for (;;) {
        // a time-sliced launch takes no new sample once its quantum is spent
        if (threadIdx.x == 0) next = (deadline && tick() >= deadline) ? a.n : atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t i = next;
        __syncthreads();
        if (i >= a.n) return;
        const DevDesc d = a.descs[i];
        run_sample<NSEL, ROWW, SPARSE, CENSUS>(a, d, lds, deadline);
    }
}

#if RSA_TU_WAVES == 0
__global__ void rsa_reset_queues(uint32_t *queues, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) queues[i] = 0;
}

// Before a time-sliced launch: every result reads "not run" until a
// workgroup reaches its sample, a sample listed for the first time starts
// from the empty lattice, and the work-queue counters restart at 0.
__global__ void rsa_prepare_launch(const DevDesc *descs, uint32_t n, DevResult *res, uint32_t *queues,
                                   uint32_t nq)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nq) queues[i] = 0;
    if (i >= n) return;
    res[i].status = kStatusNotRun;
    const DevDesc d = descs[i];
    if (d.flags & kDescFresh) {
        SampleState *st = (SampleState *)((uint8_t *)d.slab + slab_layout(d.L, d.k, d.compressed != 0).state);
        st->phase = 0;
    }
}
#endif

}  // namespace rsa

// Host-visible launch table of this translation unit:
// [row words per lane 1 or 8][dense, sparse][without, with contact census]
// for one wave count.  The library compiles this file once per wave-count
// index (RSA_TU_WAVES = 0 .. kNumWaveTiles - 1) so that the instantiations
// build in parallel.
#define RSA_CAT2(a, b) a##b
#define RSA_CAT(a, b) RSA_CAT2(a, b)
#define RSA_TABLE RSA_CAT(kPersistentKernelsW, RSA_TU_WAVES)
#define RSA_KP(ROWW, SPARSE, CENSUS) \
    (const void *)&rsa_persistent<kTileWaves[RSA_TU_WAVES], ROWW, SPARSE, CENSUS>
namespace rsa {
extern const void *RSA_TABLE[2][2][2];
const void *RSA_TABLE[2][2][2] = {
    {{RSA_KP(1, false, false), RSA_KP(1, false, true)}, {RSA_KP(1, true, false), RSA_KP(1, true, true)}},
    {{RSA_KP(8, false, false), RSA_KP(8, false, true)}, {RSA_KP(8, true, false), RSA_KP(8, true, true)}}};
#if RSA_TU_WAVES == 0
extern const void *kResetKernel;
extern const void *kPrepareKernel;
const void *kResetKernel = (const void *)&rsa_reset_queues;
const void *kPrepareKernel = (const void *)&rsa_prepare_launch;
#endif
}  // namespace rsa
