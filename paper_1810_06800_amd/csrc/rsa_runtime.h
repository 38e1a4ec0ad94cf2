// rsa_runtime.h -- internal host runtime shared by the batch entry points
// (rsa_capi.hip) and the request server (rsa_server.hip).  Not part of the C
// ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/rsa.h"
#include "rsa_device.h"

namespace rsa {
// launch tables of the kernel translation units, one per wave count
extern const void *kPersistentKernelsW0[2][2][2];
extern const void *kPersistentKernelsW1[2][2][2];
extern const void *kPersistentKernelsW2[2][2][2];
extern const void *kPersistentKernelsW3[2][2][2];
extern const void *kPersistentKernelsW4[2][2][2];
extern const void *kResetKernel;
extern const void *kPrepareKernel;
static_assert(kNumWaveTiles == 5, "one launch table per wave count");

// persistent kernel of a schedule: (wave-count index, rows wider than 64
// words, sparse clear, contact census compiled in)
const void *persistent_kernel(int waves, int wide, int sparse, int census);
// Kernel variants per wave count: wide x sparse x census.
constexpr int kKernelVariants = 8;
inline int kernel_key(int waves, int wide, int sparse, int census)
{
    return ((waves * 2 + wide) * 2 + sparse) * 2 + census;
}
}  // namespace rsa

static_assert(sizeof(rsa_result_t) == sizeof(rsa::DevResult), "result layout");
static_assert(sizeof(rsa_result_t) == 104, "result size");
static_assert(sizeof(rsa_sample_t) == 24, "sample size");

namespace rsa {

constexpr int kPlainStreams = 4;

struct Group {
    int key;                 // kernel_key of the instantiation
    int pass;                // 0 = the runs, 1 = reruns for cluster sizes
    int waves;               // index into kTileWaves
    int wide;                // rows of more than 64 words (L > 4096)
    int sparse;              // clear mode
    int census;              // contact census compiled in
    uint32_t first, count;   // range in the planned descriptor array
    uint32_t grid;
    uint32_t lds;
    size_t stride;           // slab bytes per resident workgroup
    size_t slab_off;         // offset of this group's slabs in the batch allocation
};

struct Block {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct Batch {
    uint64_t id = 0;
    uint32_t n = 0;
    Block mem;
    DevDesc *h_desc = nullptr;      // pinned
    rsa_result_t *h_res = nullptr;  // pinned
    size_t h_desc_bytes = 0, h_res_bytes = 0;
    hipEvent_t ev_start = nullptr, ev_end = nullptr, ev_done = nullptr;
    std::vector<Group> groups;
    int mode = RSA_MODE_BATCHED;
    unsigned long long *d_prof = nullptr;   // inside mem, or null
    unsigned long long *d_hist = nullptr;   // cluster-size histograms, inside mem, or null
};

struct GraphEntry {
    std::string key;
    hipGraphExec_t exec = nullptr;
};

}  // namespace rsa

struct rsa_ctx {
    int device = 0;
    int cus = 0;
    size_t lds_max = 0;
    uint64_t budget = 0;
    uint64_t held = 0;   // bytes currently allocated (in use + pooled)
    bool custom = false;
    rsa_allocator_t alloc{};
    bool poisoned = false;
    std::string last_error;
    uint64_t next_id = 1;
    std::map<uint64_t, rsa::Batch *> batches;
    std::vector<rsa::Block> pool;   // free device blocks
    std::vector<rsa::Block> pinned; // free pinned host buffers (descriptor / result staging)
    std::vector<rsa::GraphEntry> graphs;
    int64_t opt_mode = RSA_MODE_BATCHED, opt_tile = -1, opt_graph = 1, opt_slots = 0, opt_prof = 0;
    int64_t opt_ivslab = 0;
    int clock_khz = 0;
    hipStream_t plain[rsa::kPlainStreams] = {};
    hipEvent_t fork = nullptr, join[rsa::kPlainStreams] = {};
    int resident[rsa::kNumTiles][4] = {};   // cached occupancy per tile and LDS class
    std::map<std::pair<uint32_t, uint32_t>, int> tile_table;   // (L, k) -> measured best tile
    // device address of this device's static scratch array (rsa_run_batch_static),
    // looked up once per device when the first context on it is created; null
    // (with scratch_error set) if the lookup failed
    void *scratch = nullptr;
    std::string scratch_error;
};

namespace rsa {

// Records msg as the context's last error and returns code.
int fail(rsa_ctx *c, int code, const std::string &msg);
// Poisons the context after a HIP failure; returns RSA_EDEVICE.
int hip_fail(rsa_ctx *c, hipError_t e, const char *what);
bool valid_sample(const rsa_sample_t &s);
// Built-in schedule heuristic for a shape.
int default_tile(uint32_t L, uint32_t k);
// Schedule of a sample: the forced tile option, else the context's autotune
// table entry for (L, k), else the heuristic.
int sample_tile(const rsa_ctx *c, uint32_t L, uint32_t k);
// Device memory through the caller's allocator or hipMalloc, within the budget.
bool take_block(rsa_ctx *c, size_t bytes, Block &out);
void give_block(rsa_ctx *c, Block b);
// Pinned host staging from the context's pool (nullptr if hipHostMalloc fails).
void *take_pinned(rsa_ctx *c, size_t bytes);
void give_pinned(rsa_ctx *c, void *p, size_t bytes);
// Workgroups of a schedule's kernel resident on the whole device at once.
int resident_blocks(rsa_ctx *c, int tile, int wide, int sparse, int census, uint32_t lds);
// Whether a sample of a sparse-clear tile runs the interval clear: k up to
// kIntervalMaxK and at most kMaxBuckets buckets per line.  Otherwise the
// sparse clear by summary bits.
bool use_interval(uint32_t L, uint32_t k, int tile);
// Whether the interval clear's difference counts fit the workgroup's LDS
// beside the row counts (else they live in the slab).
bool interval_in_lds(uint32_t L, uint32_t k, size_t lds_max);
// The LDS bound the interval clear's difference counts are placed against:
// the device's, or 0 with RSA_OPT_IV_SLAB (counts in the slab).
size_t interval_lds_max(const rsa_ctx *c);
// Whether a sample keeps the compressed lattice (occupancy and anchor bitmaps
// instead of the int32 site map): sparse-clear tiles with k >= kCompressMinK.
bool use_compressed(uint32_t L, uint32_t k, int tile);
// Slab bytes of a sample under its tile.
size_t sample_slab(uint32_t L, uint32_t k, int tile);
// Dynamic LDS bytes the sample's kernel needs.
uint32_t sample_lds(uint32_t L, uint32_t k, int tile, size_t lds_max);
// Kernel-side descriptor of a sample; `out` is its index in the result array.
DevDesc make_dev_desc(const rsa_sample_t &s, uint32_t out, int tile, size_t lds_max);

}  // namespace rsa

#define HIP_TRY(ctx, expr)                                     \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return rsa::hip_fail(ctx, e_, #expr); \
    } while (0)

