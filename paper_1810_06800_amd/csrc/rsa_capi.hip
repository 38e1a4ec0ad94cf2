// rsa_capi.hip -- host runtime behind the C ABI of include/rsa.h.
//
// A batch is planned into groups of samples that share a schedule ("tile"),
// each group becomes one persistent launch over its own device work queue,
// and all groups of a batch run as parallel nodes of one hipGraph (instantiated
// once per launch signature and replayed).  Device memory comes from a
// per-context pool of slabs, through the caller's allocator when one is given.
#include "rsa_runtime.h"

#include <mutex>

// Static scratch of rsa_run_batch_static: work-queue counters, kernel-side
// descriptors and the per-workgroup slabs of a batch, for callers that cannot
// allocate.  Each device holds its own copy for the life of the process; host
// code reaches it only through the address hipGetSymbolAddress returns for the
// device (kept in rsa_ctx::scratch), never through this name.
static __device__ __align__(256) uint8_t scratch[RSA_STATIC_SCRATCH_BYTES];

namespace rsa {

// Kernel-side descriptors of rsa_run_batch_static travel as kernel arguments
// (the launch copies them), kStageDescs per launch, into the static scratch.
constexpr uint32_t kStageDescs = 24;
struct StageArgs {
    DevDesc d[kStageDescs];
    DevDesc *dst;
    uint32_t n;
};
static_assert(sizeof(StageArgs) <= 4096, "kernel argument size");

__global__ void rsa_stage_descs(StageArgs a)
{
    const uint32_t i = threadIdx.x;
    if (i < a.n) a.dst[i] = a.d[i];
}

// Device address of the static scratch on `device` (current), looked up once
// per device.
constexpr int kMaxScratchDevices = 64;
static void *g_scratch[kMaxScratchDevices];
static std::mutex g_scratch_mu;

static void *scratch_address(int device, std::string &err)
{
    if (device < 0 || device >= kMaxScratchDevices) {
        err = "device index beyond the scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch[device] = p;
    }
    return g_scratch[device];
}

const void *persistent_kernel(int waves, int wide, int sparse, int census)
{
    static const void *(*const tables[kNumWaveTiles])[2][2] = {
        kPersistentKernelsW0, kPersistentKernelsW1, kPersistentKernelsW2, kPersistentKernelsW3,
        kPersistentKernelsW4};
    return tables[waves][wide][sparse][census];
}

int fail(rsa_ctx *c, int code, const std::string &msg)
{
    if (c) c->last_error = msg;
    return code;
}

int hip_fail(rsa_ctx *c, hipError_t e, const char *what)
{
    if (c) {
        c->poisoned = true;
        c->last_error = std::string(what) + ": " + hipGetErrorString(e);
    }
    return RSA_EDEVICE;
}

bool valid_sample(const rsa_sample_t &s)
{
    const uint32_t known = RSA_FLAG_H_ONLY | RSA_FLAG_TRACK_CLUSTERS | RSA_FLAG_CONTACTS | RSA_FLAG_CLUSTER_SIZES;
    return s.k >= 1 && s.k <= s.L && s.L <= 32768 && (s.flags & ~known) == 0;
}

// Schedule heuristic: waves that share the select/clear of one sample grow
// with the k x k block a deposit clears; 8-row bitmap tiles and 8-row map
// tiles keep a k-row block to about k/8 cache lines.
int default_tile(uint32_t L, uint32_t k)
{
    (void)L;
    int waves = k <= 64 ? 0 : (k <= 128 ? 1 : (k <= 256 ? 2 : 3));
    return make_tile(waves, 3, 3, k >= 512 ? 1 : 0);
}

int sample_tile(const rsa_ctx *c, uint32_t L, uint32_t k)
{
    if (c->opt_tile >= 0) return (int)c->opt_tile;
    auto it = c->tile_table.find({L, k});
    return it != c->tile_table.end() ? it->second : default_tile(L, k);
}

// Relative cost of a sample: deposits (about 0.7 L^2 / k) times the words a
// deposit clears spread over the tile's waves, plus a per-step latency floor.
double sample_cost(uint32_t L, uint32_t k, int tile)
{
    double steps = 0.7 * (double)L * L / k;
    double words = (double)k * ((double)k / 64.0 + 1.0);
    return steps * (8.0 + words / (64.0 * kTileWaves[tile_waves(tile)]));
}

void *dev_alloc(rsa_ctx *c, size_t bytes)
{
    if (c->custom) return c->alloc.alloc(bytes, c->alloc.user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(rsa_ctx *c, void *p, size_t bytes)
{
    if (!p) return;
    if (c->custom)
        c->alloc.free(p, bytes, c->alloc.user);
    else
        (void)hipFree(p);
}

// Best-fit block from the pool, else a fresh allocation within the budget.
bool take_block(rsa_ctx *c, size_t bytes, Block &out)
{
    int best = -1;
    for (size_t i = 0; i < c->pool.size(); ++i) {
        size_t b = c->pool[i].bytes;
        if (b >= bytes && b <= bytes + bytes / 4 && (best < 0 || b < c->pool[best].bytes)) best = (int)i;
    }
    if (best >= 0) {
        out = c->pool[best];
        c->pool.erase(c->pool.begin() + best);
        return true;
    }
    // release pooled blocks until the new one fits the budget
    while (c->held + bytes > c->budget && !c->pool.empty()) {
        Block b = c->pool.back();
        c->pool.pop_back();
        dev_free(c, b.ptr, b.bytes);
        c->held -= b.bytes;
    }
    if (c->held + bytes > c->budget) return false;
    void *p = dev_alloc(c, bytes);
    if (!p) {
        // the caller's allocator or the device is out of memory: free the pool and retry
        while (!c->pool.empty()) {
            Block b = c->pool.back();
            c->pool.pop_back();
            dev_free(c, b.ptr, b.bytes);
            c->held -= b.bytes;
        }
        p = dev_alloc(c, bytes);
        if (!p) return false;
    }
    c->held += bytes;
    out.ptr = p;
    out.bytes = bytes;
    return true;
}

void give_block(rsa_ctx *c, Block b)
{
    if (b.ptr) c->pool.push_back(b);
}

void *take_pinned(rsa_ctx *c, size_t bytes)
{
    int best = -1;
    for (size_t i = 0; i < c->pinned.size(); ++i) {
        const size_t b = c->pinned[i].bytes;
        if (b >= bytes && b <= 2 * bytes + 4096 && (best < 0 || b < c->pinned[best].bytes)) best = (int)i;
    }
    if (best >= 0) {
        void *p = c->pinned[best].ptr;
        c->pinned.erase(c->pinned.begin() + best);
        return p;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
}

void give_pinned(rsa_ctx *c, void *p, size_t bytes)
{
    if (!p) return;
    if (c->pinned.size() >= 16) {   // keep a few for the next batches
        (void)hipHostFree(c->pinned.front().ptr);
        c->pinned.erase(c->pinned.begin());
    }
    c->pinned.push_back(Block{p, bytes});
}

int resident_blocks(rsa_ctx *c, int tile, int wide, int sparse, int census, uint32_t lds)
{
    int nb = 0;
    int threads = 64 * (kTileWaves[tile] + 1);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persistent_kernel(tile, wide, sparse, census), threads,
                                                     lds) !=
            hipSuccess ||
        nb < 1)
        nb = 1;
    return nb * c->cus;
}

bool use_interval(uint32_t L, uint32_t k, int tile) { return tile_sparse(tile) && interval_shape(L, k); }

bool interval_in_lds(uint32_t L, uint32_t k, size_t lds_max)
{
    return (size_t)lds_layout(L).total + interval_lds_bytes(k) + 64 <= lds_max;
}

size_t interval_lds_max(const rsa_ctx *c) { return c->opt_ivslab ? 0 : c->lds_max; }

bool use_compressed(uint32_t L, uint32_t k, int tile)
{
    (void)L;
    return tile_sparse(tile) && k >= kCompressMinK;
}

size_t sample_slab(uint32_t L, uint32_t k, int tile) { return slab_layout(L, k, use_compressed(L, k, tile)).total; }

uint32_t sample_lds(uint32_t L, uint32_t k, int tile, size_t lds_max)
{
    return lds_layout(L).total +
           (use_interval(L, k, tile) && interval_in_lds(L, k, lds_max) ? interval_lds_bytes(k) : 0u);
}

DevDesc make_dev_desc(const rsa_sample_t &s, uint32_t out, int tile, size_t lds_max)
{
    DevDesc d;
    std::memset(&d, 0, sizeof(d));
    d.L = s.L;
    d.k = s.k;
    d.seed = s.seed;
    d.sample = s.sample;
    d.flags = s.flags;
    d.out = out;
    d.wd = (s.L + 63) / 64;
    d.fL = make_fastdiv(s.L);
    d.fk = make_fastdiv(s.k);
    d.fC = make_fastdiv(2 * s.k + 2);
    d.fwd = make_fastdiv(d.wd);
    d.fwp = make_fastdiv(padded_words(s.L));
    d.fB = make_fastdiv(s.k + 1);
    d.interval = use_interval(s.L, s.k, tile) ? 1u : 0u;
    d.ivg = d.interval && !interval_in_lds(s.L, s.k, lds_max) ? 1u : 0u;
    d.compressed = use_compressed(s.L, s.k, tile) ? 1u : 0u;
    d.tile = (uint32_t)tile;
    d.sparse = (uint32_t)tile_sparse(tile);
    d.lg_tr = (uint32_t)tile_lg_tr(tile);
    d.lg_mr = (uint32_t)tile_lg_mr(tile);
    // read-ahead window: as many rows as two (eight for wide rows) words per
    // lane hold, a power of two, at most 16
    uint32_t budget = 64u * (s.L > 4096 ? 8u : 2u) / d.wd;
    uint32_t nr = 1;
    while (nr * 2 <= budget && nr * 2 <= 16) nr *= 2;
    d.spec_rows = nr;
    return d;
}

void destroy_batch(rsa_ctx *c, Batch *b)
{
    if (!b) return;
    if (b->ev_start) (void)hipEventDestroy(b->ev_start);
    if (b->ev_end) (void)hipEventDestroy(b->ev_end);
    if (b->ev_done) (void)hipEventDestroy(b->ev_done);
    give_pinned(c, b->h_desc, b->h_desc_bytes);
    give_pinned(c, b->h_res, b->h_res_bytes);
    give_block(c, b->mem);
    delete b;
}

hipGraphExec_t cached_graph(rsa_ctx *c, const std::string &key)
{
    for (auto &g : c->graphs)
        if (g.key == key) return g.exec;
    return nullptr;
}

}  // namespace rsa

using namespace rsa;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *rsa_strerror(int code)
{
    switch (code) {
    case RSA_OK: return "ok";
    case RSA_EINVAL: return "invalid argument";
    case RSA_ENOMEM: return "device memory budget exhausted";
    case RSA_EDEVICE: return "HIP device error";
    case RSA_ENOTREADY: return "batch not finished";
    case RSA_EBUSY: return "resource busy";
    case RSA_ENOTFOUND: return "unknown batch id";
    default: return "unknown status";
    }
}

const char *rsa_last_error(rsa_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

size_t rsa_footprint_bytes(uint32_t L, uint32_t k)
{
    if (k < 1 || k > L || L > 32768) return 0;
    return sample_slab(L, k, default_tile(L, k));
}

int rsa_num_tiles(void) { return kNumTiles; }

int rsa_tile_for_shape(uint32_t L, uint32_t k)
{
    if (k < 1 || k > L || L > 32768) return RSA_EINVAL;
    return default_tile(L, k);
}

int rsa_set_tile_table(rsa_ctx *c, const uint32_t *L, const uint32_t *k, const int32_t *tile, uint32_t n)
{
    if (!c || (n > 0 && (!L || !k || !tile))) return RSA_EINVAL;
    std::map<std::pair<uint32_t, uint32_t>, int> t;
    for (uint32_t i = 0; i < n; ++i) {
        if (k[i] < 1 || k[i] > L[i] || L[i] > 32768 || tile[i] < 0 || tile[i] >= kNumTiles)
            return fail(c, RSA_EINVAL, "bad tile table entry " + std::to_string(i));
        t[{L[i], k[i]}] = tile[i];
    }
    c->tile_table.swap(t);
    return RSA_OK;
}

int rsa_tile_for_sample(rsa_ctx *c, uint32_t L, uint32_t k)
{
    if (!c || k < 1 || k > L || L > 32768) return RSA_EINVAL;
    return sample_tile(c, L, k);
}

int rsa_tile_shape(int tile, int *waves, int *bitmap_tile_rows, int *map_tile_rows, int *sparse)
{
    if (tile < 0 || tile >= kNumTiles) return RSA_EINVAL;
    if (waves) *waves = kTileWaves[tile_waves(tile)];
    if (bitmap_tile_rows) *bitmap_tile_rows = 1 << tile_lg_tr(tile);
    if (map_tile_rows) *map_tile_rows = 1 << tile_lg_mr(tile);
    if (sparse) *sparse = tile_sparse(tile);
    return RSA_OK;
}

int rsa_create(rsa_ctx **out, int device, uint64_t hbm_budget_bytes, const rsa_allocator_t *alloc)
{
    if (!out) return RSA_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RSA_EINVAL;
    if (alloc && (!alloc->alloc || !alloc->free)) return RSA_EINVAL;
    rsa_ctx *c = new (std::nothrow) rsa_ctx();
    if (!c) return RSA_ENOMEM;
    c->device = device;
    if (alloc) {
        c->custom = true;
        c->alloc = *alloc;
    }
    hipDeviceProp_t p;
    if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&p, device) != hipSuccess) {
        delete c;
        return RSA_EDEVICE;
    }
    c->cus = p.multiProcessorCount;
    if (hipDeviceGetAttribute(&c->clock_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess)
        c->clock_khz = 0;
    c->lds_max = p.sharedMemPerBlock;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)p.totalGlobalMem);
    for (int t = 0; t < kNumWaveTiles; ++t) {
        for (int w = 0; w < 2; ++w) {
            for (int sp = 0; sp < 2; ++sp) {
                for (int cs = 0; cs < 2; ++cs) {
                    if (hipFuncSetAttribute(persistent_kernel(t, w, sp, cs),
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)(c->lds_max - 64)) != hipSuccess) {
                        delete c;
                        return RSA_EDEVICE;
                    }
                }
            }
        }
    }
    for (int i = 0; i < kPlainStreams; ++i) {
        if (hipStreamCreateWithFlags(&c->plain[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming) != hipSuccess) {
            delete c;
            return RSA_EDEVICE;
        }
    }
    if (hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return RSA_EDEVICE;
    }
    // the device is current: look up its static scratch (only
    // rsa_run_batch_static needs it, which reports a failure here)
    c->scratch = scratch_address(device, c->scratch_error);
    *out = c;
    return RSA_OK;
}

int rsa_set_option(rsa_ctx *c, int option, int64_t value)
{
    if (!c) return RSA_EINVAL;
    switch (option) {
    case RSA_OPT_MODE:
        if (value != RSA_MODE_BATCHED && value != RSA_MODE_PLAIN) return fail(c, RSA_EINVAL, "bad mode");
        c->opt_mode = value;
        return RSA_OK;
    case RSA_OPT_TILE:
        if (value < -1 || value >= kNumTiles) return fail(c, RSA_EINVAL, "bad tile");
        c->opt_tile = value;
        return RSA_OK;
    case RSA_OPT_GRAPH:
        if (value != 0 && value != 1) return fail(c, RSA_EINVAL, "bad graph flag");
        c->opt_graph = value;
        return RSA_OK;
    case RSA_OPT_SLOTS:
        if (value < 0) return fail(c, RSA_EINVAL, "bad slot bound");
        c->opt_slots = value;
        return RSA_OK;
    case RSA_OPT_PROFILE:
        if (value != 0 && value != 1) return fail(c, RSA_EINVAL, "bad profile flag");
        c->opt_prof = value;
        return RSA_OK;
    case RSA_OPT_IV_SLAB:
        if (value != 0 && value != 1) return fail(c, RSA_EINVAL, "bad interval-slab flag");
        c->opt_ivslab = value;
        return RSA_OK;
    default: return fail(c, RSA_EINVAL, "unknown option");
    }
}

int rsa_get_option(rsa_ctx *c, int option, int64_t *value)
{
    if (!c || !value) return RSA_EINVAL;
    switch (option) {
    case RSA_OPT_MODE: *value = c->opt_mode; return RSA_OK;
    case RSA_OPT_TILE: *value = c->opt_tile; return RSA_OK;
    case RSA_OPT_GRAPH: *value = c->opt_graph; return RSA_OK;
    case RSA_OPT_SLOTS: *value = c->opt_slots; return RSA_OK;
    case RSA_OPT_PROFILE: *value = c->opt_prof; return RSA_OK;
    case RSA_OPT_IV_SLAB: *value = c->opt_ivslab; return RSA_OK;
    default: return fail(c, RSA_EINVAL, "unknown option");
    }
}

int rsa_run_batch(rsa_ctx *c, const rsa_sample_t *s, uint32_t n, void *hip_stream, uint64_t *batch_id)
{
    if (!c || !batch_id || (n > 0 && !s)) return fail(c, RSA_EINVAL, "null argument");
    if (c->poisoned) return fail(c, RSA_EDEVICE, "context poisoned by an earlier device error");
    for (uint32_t i = 0; i < n; ++i)
        if (!valid_sample(s[i]))
            return fail(c, RSA_EINVAL, "invalid descriptor at index " + std::to_string(i));
    hipStream_t stream = (hipStream_t)hip_stream;
    HIP_TRY(c, hipSetDevice(c->device));

    std::unique_ptr<Batch> b(new Batch());
    b->n = n;
    b->mode = (int)c->opt_mode;

    // ---- plan: group by tile, longest samples first inside a group.
    // Entries 0..n-1 are the runs; a sample with RSA_FLAG_CLUSTER_SIZES gets a
    // second-pass entry after them (rerun to its first wrap, then histogram).
    // Group key: (pass, wave count, rows wider than 64 words, clear mode,
    // statistics compiled in) -> kernel.
    std::vector<int> tiles(n);
    std::vector<uint32_t> ent_sample, ent_pass;
    std::vector<int> keys;
    for (uint32_t i = 0; i < n; ++i) {
        tiles[i] = sample_tile(c, s[i].L, s[i].k);
        ent_sample.push_back(i);
        ent_pass.push_back(0);
        keys.push_back(kernel_key(tile_waves(tiles[i]), s[i].L > 4096 ? 1 : 0, tile_sparse(tiles[i]),
                                  (s[i].flags & RSA_FLAG_CONTACTS) ? 1 : 0));
    }
    for (uint32_t i = 0; i < n; ++i) {
        if (!(s[i].flags & RSA_FLAG_CLUSTER_SIZES)) continue;
        ent_sample.push_back(i);
        ent_pass.push_back(1);
        keys.push_back(kernel_key(tile_waves(tiles[i]), s[i].L > 4096 ? 1 : 0, tile_sparse(tiles[i]), 1));
    }
    const uint32_t ne = (uint32_t)ent_sample.size();
    const bool sizes = ne > n;
    std::vector<uint32_t> order(ne);
    for (uint32_t i = 0; i < ne; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t bb) {
        if (ent_pass[a] != ent_pass[bb]) return ent_pass[a] < ent_pass[bb];
        if (keys[a] != keys[bb]) return keys[a] > keys[bb];
        const rsa_sample_t &x = s[ent_sample[a]], &y = s[ent_sample[bb]];
        return sample_cost(x.L, x.k, tiles[ent_sample[a]]) > sample_cost(y.L, y.k, tiles[ent_sample[bb]]);
    });
    size_t total = 0;
    const size_t nq_batched = (size_t)2 * kKernelVariants * kNumWaveTiles;   // per pass and kernel
    const size_t desc_bytes = align256((size_t)std::max<uint32_t>(ne, 1) * sizeof(DevDesc));
    const size_t res_bytes = align256((size_t)std::max<uint32_t>(n, 1) * sizeof(DevResult));
    const size_t queue_count = b->mode == RSA_MODE_PLAIN ? std::max<uint32_t>(n, 1) + nq_batched : nq_batched;
    const size_t queue_bytes = align256(queue_count * 4);
    const size_t prof_words = c->opt_prof ? (size_t)std::max<uint32_t>(n, 1) * kProfSlots : 0;
    const size_t prof_bytes = align256(prof_words * 8);
    const size_t hist_words = sizes ? (size_t)n * kSizeBins : 0;
    const size_t hist_bytes = align256(hist_words * 8);
    total = desc_bytes + res_bytes + queue_bytes + prof_bytes + hist_bytes;
    for (uint32_t i = 0; i < ne;) {
        Group g;
        g.key = keys[order[i]];
        g.pass = (int)ent_pass[order[i]];
        g.waves = g.key >> 3;
        g.wide = (g.key >> 2) & 1;
        g.sparse = (g.key >> 1) & 1;
        g.census = g.key & 1;
        g.first = i;
        uint32_t j = i;
        size_t stride = 0;
        uint32_t lds = 0;
        while (j < ne && keys[order[j]] == keys[order[i]] && ent_pass[order[j]] == ent_pass[order[i]]) {
            const rsa_sample_t &x = s[ent_sample[order[j]]];
            stride = std::max(stride, sample_slab(x.L, x.k, tiles[ent_sample[order[j]]]));
            lds = std::max(lds, sample_lds(x.L, x.k, tiles[ent_sample[order[j]]], interval_lds_max(c)));
            ++j;
        }
        g.count = j - i;
        g.stride = stride;
        g.lds = lds;
        if (lds + 64 > c->lds_max) return fail(c, RSA_EINVAL, "lattice too large for LDS");
        uint32_t grid;
        if (b->mode == RSA_MODE_PLAIN && g.pass == 0) {
            grid = kPlainStreams;   // one slab per stream: samples on a stream run in order
        } else {
            grid = std::min<uint32_t>(g.count, (uint32_t)resident_blocks(c, g.waves, g.wide, g.sparse, g.census, lds));
            if (c->opt_slots > 0) grid = std::min<uint32_t>(grid, (uint32_t)c->opt_slots);
        }
        g.grid = grid;
        b->groups.push_back(g);
        i = j;
    }
    // fit the slabs into the budget, shrinking the widest groups first
    auto slab_total = [&]() {
        size_t t = 0;
        for (auto &g : b->groups) t += g.stride * g.grid;
        return t;
    };
    while (total + slab_total() > c->budget) {
        Group *big = nullptr;
        if (b->mode != RSA_MODE_PLAIN)
            for (auto &g : b->groups)
                if (g.grid > 1 && (!big || g.stride * g.grid > big->stride * big->grid)) big = &g;
        if (!big) return fail(c, RSA_ENOMEM, "batch does not fit the device memory budget");
        big->grid = std::max<uint32_t>(1, big->grid / 2);
    }
    // the second pass starts after the first has finished, so its groups
    // reuse the first pass's slabs where they are large enough
    std::vector<Group *> pass0, pass1;
    for (auto &g : b->groups) (g.pass ? pass1 : pass0).push_back(&g);
    const size_t slab_base = total;
    for (auto *g : pass0) {
        g->slab_off = total;
        total += g->stride * g->grid;
    }
    {
        size_t off = slab_base;
        for (auto *g : pass1) {
            g->slab_off = off;
            off += g->stride * g->grid;
        }
        total = std::max(total, off);
    }
    if (total > c->budget) return fail(c, RSA_ENOMEM, "batch does not fit the device memory budget");
    if (!take_block(c, total, b->mem)) return fail(c, RSA_ENOMEM, "device allocation failed");
    uint8_t *base = (uint8_t *)b->mem.ptr;
    DevDesc *d_desc = (DevDesc *)base;
    DevResult *d_res = (DevResult *)(base + desc_bytes);
    uint32_t *d_queue = (uint32_t *)(base + desc_bytes + res_bytes);
    b->d_prof = prof_words ? (unsigned long long *)(base + desc_bytes + res_bytes + queue_bytes) : nullptr;
    b->d_hist = hist_words ? (unsigned long long *)(base + desc_bytes + res_bytes + queue_bytes + prof_bytes)
                           : nullptr;

    // ---- descriptors (pinned staging), copied before the call returns
    b->h_desc = (DevDesc *)take_pinned(c, desc_bytes);
    b->h_desc_bytes = desc_bytes;
    b->h_res = (rsa_result_t *)take_pinned(c, res_bytes);
    b->h_res_bytes = res_bytes;
    if (!b->h_desc || !b->h_res) {
        destroy_batch(c, b.release());
        return fail(c, RSA_ENOMEM, "pinned host allocation failed");
    }
    for (uint32_t i = 0; i < ne; ++i) {
        const uint32_t si = ent_sample[order[i]];
        b->h_desc[i] = make_dev_desc(s[si], si, tiles[si], interval_lds_max(c));
        if (ent_pass[order[i]]) b->h_desc[i].flags |= kDescSizesPass;
    }
    HIP_TRY(c, hipEventCreate(&b->ev_start));
    HIP_TRY(c, hipEventCreate(&b->ev_end));
    HIP_TRY(c, hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming));
    if (ne > 0)
        HIP_TRY(c, hipMemcpyAsync(d_desc, b->h_desc, (size_t)ne * sizeof(DevDesc),
                                  hipMemcpyHostToDevice, stream));

    // ---- launches
    if (b->d_prof) {
        // zero the counters with the fill kernel (outside any graph)
        uint32_t words = (uint32_t)(prof_words * 2);
        uint32_t *pw = (uint32_t *)b->d_prof;
        void *zargs[] = {&pw, &words};
        HIP_TRY(c, hipLaunchKernel(kResetKernel, dim3((words + 255) / 256), dim3(256), zargs, 0, stream));
    }
    if (b->d_hist) {
        // histograms of samples without the flag read as zero
        uint32_t words = (uint32_t)(hist_words * 2);
        uint32_t *hw = (uint32_t *)b->d_hist;
        void *zargs[] = {&hw, &words};
        HIP_TRY(c, hipLaunchKernel(kResetKernel, dim3((words + 255) / 256), dim3(256), zargs, 0, stream));
    }
    HIP_TRY(c, hipEventRecord(b->ev_start, stream));
    // queue counters: the plain form's per-sample counters first, then one
    // per (pass, kernel) for the persistent launches
    const size_t qbase = b->mode == RSA_MODE_PLAIN ? std::max<uint32_t>(n, 1) : 0;
    std::vector<KernelArgs> args;
    for (auto &g : b->groups) {
        KernelArgs a{};
        a.descs = d_desc + g.first;
        a.n = g.count;
        a.tile = (uint32_t)g.waves;
        a.queue = d_queue + qbase + (size_t)g.pass * kKernelVariants * kNumWaveTiles + g.key;
        a.slabs = base + g.slab_off;
        a.slab_stride = g.stride;
        a.results = d_res;
        a.prof = g.pass ? nullptr : b->d_prof;   // counters describe the runs, not the reruns
        a.hist = b->d_hist;
        args.push_back(a);
    }
    uint32_t nq = (uint32_t)queue_count;
    void *rargs[] = {&d_queue, &nq};
    const dim3 rgrid((nq + 255) / 256), rblock(256);
    if (n == 0) {
        // nothing to run
    } else if (b->mode == RSA_MODE_PLAIN) {
        // one launch per sample, round-robin over four streams forked from
        // the caller's stream; one slab per stream.  Second-pass groups run
        // afterwards as persistent launches on the caller's stream.
        HIP_TRY(c, hipLaunchKernel(kResetKernel, rgrid, rblock, rargs, 0, stream));
        HIP_TRY(c, hipEventRecord(c->fork, stream));
        for (int i = 0; i < kPlainStreams; ++i) HIP_TRY(c, hipStreamWaitEvent(c->plain[i], c->fork, 0));
        uint32_t idx = 0;
        for (auto &g : b->groups) {
            if (g.pass) continue;
            int threads = 64 * (kTileWaves[g.waves] + 1);
            for (uint32_t j = 0; j < g.count; ++j, ++idx) {
                int si = (int)(idx % kPlainStreams);
                KernelArgs a{};
                a.descs = d_desc + g.first + j;
                a.n = 1;
                a.tile = (uint32_t)g.waves;
                a.queue = d_queue + g.first + j;
                a.slabs = base + g.slab_off + (size_t)si * g.stride;
                a.slab_stride = 0;
                a.results = d_res;
                a.prof = b->d_prof;
                a.hist = b->d_hist;
                void *kargs[] = {&a};
                HIP_TRY(c, hipLaunchKernel(persistent_kernel(g.waves, g.wide, g.sparse, g.census), dim3(1),
                                           dim3(threads), kargs, g.lds, c->plain[si]));
            }
        }
        for (int i = 0; i < kPlainStreams; ++i) {
            HIP_TRY(c, hipEventRecord(c->join[i], c->plain[i]));
            HIP_TRY(c, hipStreamWaitEvent(stream, c->join[i], 0));
        }
        for (size_t i = 0; i < args.size(); ++i) {
            const Group &g = b->groups[i];
            if (!g.pass) continue;
            void *kargs[] = {&args[i]};
            HIP_TRY(c, hipLaunchKernel(persistent_kernel(g.waves, g.wide, g.sparse, g.census), dim3(g.grid),
                                       dim3(64 * (kTileWaves[g.waves] + 1)), kargs, g.lds, stream));
        }
    } else {
        // one graph: reset the queues, every first-pass group's persistent
        // launch side by side, then the second-pass groups after all of them
        std::string key;
        key.reserve(64 * args.size());
        for (size_t i = 0; i < args.size(); ++i) {
            const Group &g = b->groups[i];
            char buf[64];
            std::snprintf(buf, sizeof(buf), "%d:%d:%u:%u|", g.pass, g.key, g.grid, g.lds);
            key += buf;
            key.append((const char *)&args[i], sizeof(KernelArgs));
        }
        if (c->opt_graph) {
            hipGraphExec_t exec = cached_graph(c, key);
            if (!exec) {
                hipGraph_t graph;
                HIP_TRY(c, hipGraphCreate(&graph, 0));
                hipGraphNode_t reset;
                hipKernelNodeParams rp;
                std::memset(&rp, 0, sizeof(rp));
                rp.func = (void *)kResetKernel;
                rp.gridDim = rgrid;
                rp.blockDim = rblock;
                rp.kernelParams = rargs;
                HIP_TRY(c, hipGraphAddKernelNode(&reset, graph, nullptr, 0, &rp));
                std::vector<hipGraphNode_t> first;
                for (int pass = 0; pass < 2; ++pass) {
                    for (size_t i = 0; i < args.size(); ++i) {
                        const Group &g = b->groups[i];
                        if (g.pass != pass) continue;
                        hipKernelNodeParams kp;
                        std::memset(&kp, 0, sizeof(kp));
                        void *kargs[] = {&args[i]};
                        kp.func = (void *)persistent_kernel(g.waves, g.wide, g.sparse, g.census);
                        kp.gridDim = dim3(g.grid);
                        kp.blockDim = dim3(64 * (kTileWaves[g.waves] + 1));
                        kp.sharedMemBytes = g.lds;
                        kp.kernelParams = kargs;
                        hipGraphNode_t node;
                        if (pass == 0) {
                            HIP_TRY(c, hipGraphAddKernelNode(&node, graph, &reset, 1, &kp));
                            first.push_back(node);
                        } else {
                            HIP_TRY(c, hipGraphAddKernelNode(&node, graph, first.data(), first.size(), &kp));
                        }
                    }
                }
                hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
                if (c->graphs.size() >= 8) {
                    (void)hipGraphExecDestroy(c->graphs.front().exec);
                    c->graphs.erase(c->graphs.begin());
                }
                c->graphs.push_back(GraphEntry{key, exec});
            }
            HIP_TRY(c, hipGraphLaunch(exec, stream));
        } else {
            HIP_TRY(c, hipLaunchKernel(kResetKernel, rgrid, rblock, rargs, 0, stream));
            for (int pass = 0; pass < 2; ++pass) {
                for (size_t i = 0; i < args.size(); ++i) {
                    const Group &g = b->groups[i];
                    if (g.pass != pass) continue;
                    void *kargs[] = {&args[i]};
                    HIP_TRY(c, hipLaunchKernel(persistent_kernel(g.waves, g.wide, g.sparse, g.census),
                                               dim3(g.grid), dim3(64 * (kTileWaves[g.waves] + 1)), kargs,
                                               g.lds, stream));
                }
            }
        }
    }
    HIP_TRY(c, hipEventRecord(b->ev_end, stream));
    if (n > 0)
        HIP_TRY(c, hipMemcpyAsync(b->h_res, d_res, (size_t)n * sizeof(DevResult), hipMemcpyDeviceToHost,
                                  stream));
    HIP_TRY(c, hipEventRecord(b->ev_done, stream));
    b->id = c->next_id++;
    *batch_id = b->id;
    c->batches[b->id] = b.get();
    b.release();
    return RSA_OK;
}

int rsa_run_batch_static(rsa_ctx *c, const rsa_sample_t *s, uint32_t n, rsa_result_t *d_results,
                         void *hip_stream)
{
    if (!c || (n > 0 && (!s || !d_results))) return fail(c, RSA_EINVAL, "null argument");
    if (c->poisoned) return fail(c, RSA_EDEVICE, "context poisoned by an earlier device error");
    if (n > RSA_STATIC_MAX_SAMPLES)
        return fail(c, RSA_EINVAL, "rsa_run_batch_static takes at most " +
                                       std::to_string(RSA_STATIC_MAX_SAMPLES) + " samples per call");
    for (uint32_t i = 0; i < n; ++i) {
        if (!valid_sample(s[i]))
            return fail(c, RSA_EINVAL, "invalid descriptor at index " + std::to_string(i));
        if (s[i].flags & RSA_FLAG_CLUSTER_SIZES)
            return fail(c, RSA_EINVAL, "RSA_FLAG_CLUSTER_SIZES needs rsa_run_batch (index " +
                                           std::to_string(i) + ")");
    }
    if (!c->scratch) return fail(c, RSA_EDEVICE, "no static scratch on this device: " + c->scratch_error);
    if (n == 0) return RSA_OK;
    hipStream_t stream = (hipStream_t)hip_stream;
    HIP_TRY(c, hipSetDevice(c->device));

    // ---- plan on the stack: group by kernel, longest samples first inside a
    // group (the order rsa_run_batch uses), groups one after another
    uint16_t order[RSA_STATIC_MAX_SAMPLES];
    uint8_t key[RSA_STATIC_MAX_SAMPLES];
    int16_t tile[RSA_STATIC_MAX_SAMPLES];
    float cost[RSA_STATIC_MAX_SAMPLES];
    for (uint32_t i = 0; i < n; ++i) {
        tile[i] = (int16_t)sample_tile(c, s[i].L, s[i].k);
        key[i] = (uint8_t)kernel_key(tile_waves(tile[i]), s[i].L > 4096 ? 1 : 0, tile_sparse(tile[i]),
                                     (s[i].flags & RSA_FLAG_CONTACTS) ? 1 : 0);
        cost[i] = (float)sample_cost(s[i].L, s[i].k, tile[i]);
        order[i] = (uint16_t)i;
    }
    std::sort(order, order + n, [&](uint16_t a, uint16_t b) {
        if (key[a] != key[b]) return key[a] > key[b];
        if (cost[a] != cost[b]) return cost[a] > cost[b];
        return a < b;
    });
    // scratch: queue counters, descriptors, then the slabs of one group at a time
    const size_t queue_bytes = 256;
    const size_t desc_bytes = align256((size_t)n * sizeof(DevDesc));
    const size_t slab_base = queue_bytes + desc_bytes;
    uint8_t *base = (uint8_t *)c->scratch;
    uint32_t *d_queue = (uint32_t *)base;
    DevDesc *d_desc = (DevDesc *)(base + queue_bytes);
    struct StaticGroup {
        int key;
        uint32_t first, count, grid, lds;
        size_t stride;
    };
    StaticGroup groups[2 * kKernelVariants * kNumWaveTiles];
    uint32_t ng = 0;
    for (uint32_t i = 0; i < n;) {
        uint32_t j = i;
        size_t stride = 0;
        uint32_t lds = 0;
        while (j < n && key[order[j]] == key[order[i]]) {
            const rsa_sample_t &x = s[order[j]];
            stride = std::max(stride, sample_slab(x.L, x.k, tile[order[j]]));
            lds = std::max(lds, sample_lds(x.L, x.k, tile[order[j]], interval_lds_max(c)));
            ++j;
        }
        StaticGroup g;
        g.key = key[order[i]];
        g.first = i;
        g.count = j - i;
        g.stride = stride;
        g.lds = lds;
        if (lds + 64 > c->lds_max) return fail(c, RSA_EINVAL, "lattice too large for LDS");
        if (slab_base + stride > (size_t)RSA_STATIC_SCRATCH_BYTES)
            return fail(c, RSA_ENOMEM, "a sample needs " + std::to_string(stride) +
                                           " bytes of slab; the static scratch holds " +
                                           std::to_string((size_t)RSA_STATIC_SCRATCH_BYTES - slab_base) +
                                           " after the descriptors");
        const uint32_t fit = (uint32_t)(((size_t)RSA_STATIC_SCRATCH_BYTES - slab_base) / stride);
        const int waves = g.key >> 3, wide = (g.key >> 2) & 1, sparse = (g.key >> 1) & 1, census = g.key & 1;
        g.grid = std::min(std::min(g.count, fit), (uint32_t)resident_blocks(c, waves, wide, sparse, census, lds));
        if (c->opt_slots > 0) g.grid = std::min<uint32_t>(g.grid, (uint32_t)c->opt_slots);
        groups[ng++] = g;
        i = j;
    }
    // ---- launches on the caller's stream: counters zeroed by a kernel, the
    // descriptors staged through kernel arguments, then one persistent launch
    // per group in stream order (each group reuses the slab region)
    uint32_t nq = (uint32_t)(queue_bytes / 4);
    void *rargs[] = {&d_queue, &nq};
    HIP_TRY(c, hipLaunchKernel(kResetKernel, dim3(1), dim3(256), rargs, 0, stream));
    for (uint32_t i0 = 0; i0 < n; i0 += kStageDescs) {
        StageArgs sa;
        sa.n = std::min<uint32_t>(kStageDescs, n - i0);
        sa.dst = d_desc + i0;
        for (uint32_t q = 0; q < sa.n; ++q) sa.d[q] = make_dev_desc(s[order[i0 + q]], order[i0 + q], tile[order[i0 + q]], interval_lds_max(c));
        void *sargs[] = {&sa};
        HIP_TRY(c, hipLaunchKernel((const void *)&rsa_stage_descs, dim3(1), dim3(kStageDescs), sargs, 0, stream));
    }
    for (uint32_t gi = 0; gi < ng; ++gi) {
        const StaticGroup &g = groups[gi];
        const int waves = g.key >> 3, wide = (g.key >> 2) & 1, sparse = (g.key >> 1) & 1, census = g.key & 1;
        KernelArgs a{};
        a.descs = d_desc + g.first;
        a.n = g.count;
        a.tile = (uint32_t)waves;
        a.queue = d_queue + gi;
        a.slabs = base + slab_base;
        a.slab_stride = g.stride;
        a.results = (DevResult *)d_results;
        void *kargs[] = {&a};
        HIP_TRY(c, hipLaunchKernel(persistent_kernel(waves, wide, sparse, census), dim3(g.grid),
                                   dim3(64 * (kTileWaves[waves] + 1)), kargs, g.lds, stream));
    }
    return RSA_OK;
}

int rsa_results(rsa_ctx *c, uint64_t batch_id, rsa_result_t *out, uint32_t n, int wait)
{
    if (!c) return RSA_EINVAL;
    auto it = c->batches.find(batch_id);
    if (it == c->batches.end()) return fail(c, RSA_ENOTFOUND, "unknown batch id");
    Batch *b = it->second;
    if (n != b->n || (n > 0 && !out)) return fail(c, RSA_EINVAL, "result count differs from batch size");
    if (wait) {
        hipError_t e = hipEventSynchronize(b->ev_done);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    } else {
        hipError_t e = hipEventQuery(b->ev_done);
        if (e == hipErrorNotReady) return RSA_ENOTREADY;
        if (e != hipSuccess) return hip_fail(c, e, "hipEventQuery");
    }
    if (n > 0) std::memcpy(out, b->h_res, (size_t)n * sizeof(rsa_result_t));
    c->batches.erase(it);
    destroy_batch(c, b);
    return RSA_OK;
}

int rsa_batch_elapsed_ms(rsa_ctx *c, uint64_t batch_id, float *ms)
{
    if (!c || !ms) return RSA_EINVAL;
    auto it = c->batches.find(batch_id);
    if (it == c->batches.end()) return fail(c, RSA_ENOTFOUND, "unknown batch id");
    Batch *b = it->second;
    hipError_t e = hipEventSynchronize(b->ev_end);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    e = hipEventElapsedTime(ms, b->ev_start, b->ev_end);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventElapsedTime");
    return RSA_OK;
}

int rsa_batch_profile(rsa_ctx *c, uint64_t batch_id, uint64_t *out, uint32_t n, uint32_t *slots,
                      uint32_t *clock_khz)
{
    if (!c) return RSA_EINVAL;
    auto it = c->batches.find(batch_id);
    if (it == c->batches.end()) return fail(c, RSA_ENOTFOUND, "unknown batch id");
    Batch *b = it->second;
    if (slots) *slots = kProfSlots;
    if (clock_khz) *clock_khz = (uint32_t)c->clock_khz;
    if (!b->d_prof) return fail(c, RSA_EINVAL, "batch was not profiled");
    if (n != b->n || (n > 0 && !out)) return fail(c, RSA_EINVAL, "count differs from batch size");
    hipError_t e = hipEventSynchronize(b->ev_end);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    e = hipMemcpy(out, b->d_prof, (size_t)n * kProfSlots * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy");
    return RSA_OK;
}

int rsa_batch_cluster_sizes(rsa_ctx *c, uint64_t batch_id, uint64_t *out, uint32_t n)
{
    if (!c) return RSA_EINVAL;
    auto it = c->batches.find(batch_id);
    if (it == c->batches.end()) return fail(c, RSA_ENOTFOUND, "unknown batch id");
    Batch *b = it->second;
    if (!b->d_hist) return fail(c, RSA_EINVAL, "no sample of the batch asked for cluster sizes");
    if (n != b->n || (n > 0 && !out)) return fail(c, RSA_EINVAL, "count differs from batch size");
    hipError_t e = hipEventSynchronize(b->ev_end);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    e = hipMemcpy(out, b->d_hist, (size_t)n * kSizeBins * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy");
    return RSA_OK;
}

void rsa_destroy(rsa_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : c->batches) destroy_batch(c, kv.second);
    c->batches.clear();
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    for (auto &b : c->pool) dev_free(c, b.ptr, b.bytes);
    for (auto &b : c->pinned) (void)hipHostFree(b.ptr);
    for (int i = 0; i < kPlainStreams; ++i) {
        if (c->plain[i]) (void)hipStreamDestroy(c->plain[i]);
        if (c->join[i]) (void)hipEventDestroy(c->join[i]);
    }
    if (c->fork) (void)hipEventDestroy(c->fork);
    delete c;
}

}  // extern "C"
