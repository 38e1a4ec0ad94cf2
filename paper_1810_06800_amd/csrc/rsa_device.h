// rsa_device.h -- types shared by the host runtime and the gfx950 kernels of
// the k-mer RSA library (arXiv:1810.06800).  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rsa {

// Division by a run-time constant d <= 2^31 via a 32-bit multiply-high
// (Granlund and Montgomery, PLDI'94, round-up method): q = (mulhi(n, m) + n) >> l
// with l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1; exact for every
// 32-bit n.
struct FastDiv {
    uint32_t d, m, l, pad;
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
    return FastDiv{d, (uint32_t)m, l, 0};
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    uint64_t t = __umulhi(n, f.m);
    return (uint32_t)((t + n) >> f.l);
}

// Padded extents shared by every tile shape: bitmap rows of a multiple of 16
// words and a multiple of 32 rows, a site map of a multiple of 32 in both
// directions, so one slab size fits all tile shapes of a lattice.
__host__ __device__ inline uint32_t padded_words(uint32_t L) { return ((L + 63) / 64 + 15) & ~15u; }
__host__ __device__ inline uint32_t padded_side(uint32_t L) { return (L + 31) & ~31u; }
__host__ __device__ inline uint32_t summary_words(uint32_t L) { return (padded_words(L) + 63) / 64; }

// Anchor intervals (the sparse clear of long k-mers).  On one line (a row of
// H anchors, a column of V anchors) the available anchors are the intervals
// [a, b-k+1] of the empty runs [a, b] of length >= k; two of them start at
// least k+1 apart, so cut into buckets of k+1 positions the line holds at
// most one piece of an interval per bucket, ceil(L/(k+1)) buckets per line.
// A bucket entry is start | end << 16, or kNoSeg.
constexpr uint32_t kNoSeg = 0xFFFFFFFFu;
constexpr uint32_t kMaxBuckets = 64;       // one wave reads a whole line
constexpr uint32_t kIntervalMaxK = 4096;   // difference counts of a k-row block
__host__ __device__ inline uint32_t num_buckets(uint32_t L, uint32_t k) { return (L + k) / (k + 1); }
__host__ __device__ inline bool has_buckets(uint32_t L, uint32_t k) { return num_buckets(L, k) <= kMaxBuckets; }
// Compressed lattice (Sec. II.E stores a few bits per site instead of the
// cluster data): for long k-mers the int32 site map gives way to six bitmaps
// of one bit per site -- occupied by an H k-mer, by a V k-mer, H anchor, V
// anchor, the occupancies kept both along rows and along columns -- and an
// open-addressing table from a k-mer's canonical placement index to its
// deposit number.  Words hold 64 consecutive sites of one line; the copies
// written across their lines are stored 16 lines to a 128-byte tile.
constexpr uint32_t kCompressMinK = 512;
__host__ __device__ inline uint32_t line_words(uint32_t L) { return (L + 63) / 64; }
__host__ __device__ inline uint32_t tile16(uint32_t L) { return (L + 15) / 16; }
__host__ __device__ inline uint32_t hash_slots(uint32_t L, uint32_t k)
{
    const uint64_t need = 2ull * ((uint64_t)L * L / k + 1);
    uint32_t c = 64;
    while (c < need) c <<= 1;
    return c;
}

// The interval clear's per-row difference counts of a k-row block and their
// sums over 64 rows: in LDS after the common layout when they fit, else in
// the slab, two sets used by alternate steps (a set is cleared during its
// step and reused two steps later, after a wait that orders the clearing
// stores before the next use).
__host__ __device__ inline uint32_t interval_diff_words(uint32_t k) { return (k + 1 + 3) & ~3u; }
__host__ __device__ inline uint32_t interval_lds_bytes(uint32_t k) { return 4 * (interval_diff_words(k) + 68); }
__host__ __device__ inline bool interval_shape(uint32_t L, uint32_t k) { return k <= kIntervalMaxK && has_buckets(L, k); }

// One sample as the kernels see it.
struct DevDesc {
    uint32_t L, k;
    uint64_t seed;
    uint32_t sample, flags;
    uint32_t out;      // index into the result array
    uint32_t wd;       // 64-bit words per bitmap row, ceil(L/64)
    uint32_t lg_tr;    // bitmap tile: 2^lg_tr rows x 2^(4-lg_tr) words (128 B)
    uint32_t lg_mr;    // site-map tile: 2^lg_mr rows x 2^(5-lg_mr) sites (128 B)
    uint32_t spec_rows;   // rows read ahead of each clear (power of two)
    uint32_t tile;        // schedule id reported in the result
    uint32_t sparse;      // clear mode: 0 dense, 1 sparse (summary bits or intervals)
    uint32_t interval;    // sparse mode by anchor intervals (1) or by summary bits (0)
    uint32_t compressed;  // site map replaced by occupancy / anchor bitmaps (1)
    uint32_t ivg;         // interval clear with its difference counts in the slab (1) or in LDS (0)
    uint64_t slab;        // the sample's own slab, or 0 = the workgroup's slab
    FastDiv fL;        // division by L
    FastDiv fk;        // division by k
    FastDiv fC;        // division by 2k+2 (contacts per k-mer)
    FastDiv fwd;       // division by wd
    FastDiv fwp;       // division by the padded row words
    FastDiv fB;        // division by k+1 (interval bucket width)
};

// Mirrors rsa_result_t of include/rsa.h (104 bytes).
struct DevResult {
    int64_t n_jam, n_wrap_x, n_wrap_y, n_wrap_any;
    uint64_t occ_hash, seq_hash;
    int32_t n_clusters_jam, n_nonwrapping_jam;
    int32_t status, tile;
    uint64_t alg_bytes, wchg_words;
    int64_t n_contacts_x, n_contacts_y, n_contacts_xy;
};

// Fixed capacities of the per-workgroup LDS areas.
constexpr uint32_t kRing = 512;    // placements in flight between the waves
constexpr uint32_t kBatch = 64;    // deposits the labelling wave takes at once
constexpr uint32_t kEdges = 256;   // contact edges per labelling chunk
constexpr uint32_t kSlots = 640;   // local union-find slots: a batch plus two per edge
constexpr uint32_t kHash = 1024;   // open-addressing table of global roots

// LDS layout for a sample of side L (bytes from the start of dynamic LDS).
struct LdsLayout {
    uint32_t hdr, cnt0, cnt1, cnt2, ring, banc, edges, slots, hash, total;
    uint32_t n1, n2;
};

__host__ __device__ inline LdsLayout lds_layout(uint32_t L)
{
    LdsLayout s;
    uint32_t rows = 2 * L;
    s.n1 = (rows + 63) / 64;
    s.n2 = (rows + 4095) / 4096;
    uint32_t off = 0;
    const uint32_t sizes[9] = {256,                       // header
                               ((rows + 1) / 2) * 4,      // row counts, two uint16 per word
                               s.n1 * 4,                  // sums over 64 rows
                               s.n2 * 4,                  // sums over 4096 rows
                               kRing * 4, kBatch * 4, kEdges * 16, kSlots * 20, kHash * 8};
    uint32_t at[9];
    for (int i = 0; i < 9; ++i) {
        at[i] = off;
        off += (sizes[i] + 15) & ~15u;
    }
    s.hdr = at[0];
    s.cnt0 = at[1];
    s.cnt1 = at[2];
    s.cnt2 = at[3];
    s.ring = at[4];
    s.banc = at[5];
    s.edges = at[6];
    s.slots = at[7];
    s.hash = at[8];
    s.total = off;
    return s;
}

// Per-sample device state, one slab per resident workgroup (batched runs) or
// per sample (time-sliced runs):
//   avail[0], avail[1]  availability bitmaps of H / V placements: bit x%64 of
//                       word x/64 of row y is anchor (y, x); words are stored
//                       in 128-byte tiles of 2^lg_tr rows x 2^(4-lg_tr) words
//   map                 int32 site -> k-mer id (deposit number), -1 = empty,
//                       in 128-byte tiles of 2^lg_mr rows x 2^(5-lg_mr) sites
//   node                per k-mer union-find record {parent, dx, dy, meta}:
//                       (dx, dy) = anchor minus the parent's anchor, unwrapped;
//                       meta (roots only) = rank | wraps-in-x << 8 | -in-y << 9
//   kmer                per k-mer anchor site index | orientation << 31
//   sum[0], sum[1]      summary bits of the availability bitmaps, row-major:
//                       bit w%64 of word w/64 of row y is set while word w
//                       of row y may be non-zero (used by the sparse clear)
//   state               SampleState, then the LDS row counts of a sample
//                       that yielded (time-sliced runs only)
//   hb, vb              anchor-interval buckets of H rows / V columns (when
//                       has_buckets), bucket-major: entry j of line q at
//                       [j * padded_side + q]
//   ohr, ovr, ohc, ovc  compressed lattice (instead of map): H / V occupancy
//                       along rows (ovr tiled) and along columns (ohc tiled)
//   ahr, avc            H anchors along rows, V anchors along columns
//   khash               placement index + 1 | deposit number << 32, per slot
//   ivd                 two sets of the interval clear's difference counts
//                       (used when they do not fit LDS)
struct SlabLayout {
    size_t avail0, avail1, sum0, sum1, map, node, kmer, state, hb, vb;
    size_t ohr, ovr, ohc, ovc, ahr, avc, khash, ivd, total;
};

// Status values of a time-sliced run besides 0 and the negative errors:
// the sample yielded with its state saved, or was not reached in this launch.
constexpr int32_t kStatusYielded = 1;
constexpr int32_t kStatusNotRun = 2;
// Descriptor flag of a time-sliced launch, above the public flags: the
// sample has no saved state yet.
constexpr uint32_t kDescFresh = 1u << 8;
// Descriptor flag of a batch's second pass: rerun the sample up to its first
// wrap (the first pass's n_wrap_any) and histogram the cluster sizes there.
constexpr uint32_t kDescSizesPass = 1u << 9;
// Cluster-size histogram bins: bin b counts clusters of 2^b .. 2^(b+1)-1 sites.
constexpr uint32_t kSizeBins = 32;

// What a sample that yields before jamming keeps in its slab.  The bitmaps,
// map and union-find stay where they are; this record and the LDS row counts
// are all the workgroup holds besides them between two deposits.
struct SampleState {
    uint32_t phase;      // 0 not started, 1 yielded, 2 finished
    uint32_t t;          // deposits made
    uint32_t P;          // placement of deposit t, already selected
    uint32_t lab_stop;   // labelling ended early (both wrap steps known)
    int32_t nx, ny;      // first wrap steps so far (1-based) or -1
    int32_t status;
    uint32_t pad;
    uint64_t occ, seqh, wchg;
    uint64_t pad2;
    DevResult result;    // the final record once phase == 2
};
constexpr size_t kStateBytes = 256;
static_assert(sizeof(SampleState) <= kStateBytes, "state record");

__host__ __device__ inline uint32_t lds_count_bytes(uint32_t L)
{
    LdsLayout l = lds_layout(L);
    return l.ring - l.cnt0;
}

__host__ __device__ inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

__host__ __device__ inline SlabLayout slab_layout(uint32_t L, uint32_t k, bool compressed = false)
{
    SlabLayout s;
    size_t wp = padded_words(L), lp = padded_side(L);
    size_t cap = (size_t)L * L / k + 1;
    size_t off = 0;
    s.avail0 = off; off = align256(off + lp * wp * 8);
    s.avail1 = off; off = align256(off + lp * wp * 8);
    s.sum0 = off;   off = align256(off + lp * summary_words(L) * 8);   // summary bits, see below
    s.sum1 = off;   off = align256(off + lp * summary_words(L) * 8);
    s.map = off;    off = align256(off + (compressed ? 0 : lp * lp * 4));
    const size_t bw = (size_t)line_words(L) * tile16(L) * 16 * 8;   // one bitmap (tiled or not)
    const size_t nbm = compressed ? bw : 0;
    s.ohr = off;    off = align256(off + nbm);
    s.ovr = off;    off = align256(off + nbm);
    s.ohc = off;    off = align256(off + nbm);
    s.ovc = off;    off = align256(off + nbm);
    s.ahr = off;    off = align256(off + nbm);
    s.avc = off;    off = align256(off + nbm);
    s.khash = off;  off = align256(off + (compressed ? (size_t)hash_slots(L, k) * 8 : 0));
    s.node = off;   off = align256(off + cap * 16);
    s.kmer = off;   off = align256(off + cap * 4);
    s.state = off;  off = align256(off + kStateBytes + lds_count_bytes(L));
    const size_t nb = has_buckets(L, k) ? (size_t)num_buckets(L, k) * lp * 4 : 0;
    s.hb = off;     off = align256(off + nb);
    s.vb = off;     off = align256(off + nb);
    s.ivd = off;    off = align256(off + (interval_shape(L, k) ? (size_t)8 * (interval_diff_words(k) + 68) : 0));
    s.total = off;
    return s;
}

struct KernelArgs {
    const DevDesc *descs;
    uint32_t n;
    uint32_t tile;
    uint32_t *queue;
    uint8_t *slabs;
    uint64_t slab_stride;
    DevResult *results;
    unsigned long long *prof;   // kProfSlots counters per sample, or null
    uint64_t quantum;           // wall-clock ticks a workgroup runs before its
                                // sample yields; 0 = every sample to jamming
    unsigned long long *hist;   // kSizeBins per sample (by result index), or null
};

// Optional per-sample phase counters (device wall-clock ticks unless noted).
enum ProfSlot {
    kProfInit = 0,      // state initialisation
    kProfSelTotal,      // selecting wave, first step to jamming
    kProfSelRing,       // waiting for ring space
    kProfSelSelect,     // draw + hierarchical select + row read
    kProfSelClear,      // clearing blocked placements (incl. helper waits)
    kProfLabTotal,      // labelling wave, start to exit
    kProfLabIdle,       // waiting for placements
    kProfLabMap,        // site-map writes of a batch
    kProfLabGather,     // contact gathering
    kProfLabResolve,    // global finds and slot assignment
    kProfLabMerge,      // ordered merge in LDS
    kProfLabWriteBack,  // local forest written back
    kProfLabBatches,    // count
    kProfLabEdges,      // count
    kProfLabFlushes,    // count
    kProfSteps,         // count
    kProfSpecHits,      // count: next row read ahead of the clear was the right one
    kProfSelHook,       // read-ahead outside the clear (sparse clear; 0 with the dense one)
    kProfSelProcess,    // the selecting wave's clear: reads, hashes, bits, counts
    kProfIvCut,         // interval clear, selecting wave: lines cut (reads, writes, counts)
    kProfIvMeet,        // interval clear, selecting wave: waiting at the mid-step barrier
    kProfIvRows,        // interval clear, selecting wave: row counts from the cuts
    kProfSlots
};

// Schedules ("tiles"): waves that share the select/clear of one sample (one
// more wave per workgroup labels clusters), the bitmap tile height and the
// site-map tile height.  tile = waves + kNumWaveTiles * (lg_tr + 5 * lg_mr).
constexpr int kNumWaveTiles = 5;
constexpr int kTileWaves[kNumWaveTiles] = {1, 2, 3, 7, 15};   // + 1 labelling wave: <= 1024 threads
// The last dimension is the clear mode: 0 = dense (read every word of the
// blocked rectangles), 1 = sparse (read the summary bits first and only the
// words that are still non-zero).
constexpr int kNumTiles = kNumWaveTiles * 5 * 6 * 2;
__host__ __device__ inline int tile_waves(int tile) { return tile % kNumWaveTiles; }
__host__ __device__ inline int tile_lg_tr(int tile) { return (tile / kNumWaveTiles) % 5; }
__host__ __device__ inline int tile_lg_mr(int tile) { return (tile / (kNumWaveTiles * 5)) % 6; }
__host__ __device__ inline int tile_sparse(int tile) { return tile / (kNumWaveTiles * 5 * 6); }
__host__ __device__ inline int make_tile(int waves, int lg_tr, int lg_mr, int sparse = 0)
{
    return waves + kNumWaveTiles * (lg_tr + 5 * (lg_mr + 6 * sparse));
}

}  // namespace rsa
