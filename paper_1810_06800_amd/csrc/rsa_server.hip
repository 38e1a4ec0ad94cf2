// rsa_server.hip -- request server behind the C ABI of include/rsa.h:
// continuous batching of independent RSA runs (Sec. II.A) that arrive over
// time.
//
// Requests queue on the host.  A queued sample is admitted, oldest request
// first, once a resident slot and arena space for its slab are free; its
// lattice then stays in HBM until it jams.  The device runs time-sliced
// launches of the persistent kernels: a workgroup takes samples from its
// group's list until its quantum is spent, and a sample still running then
// saves its row counts and chain position in its slab and yields (the
// kernel's SampleState); the next launch lists it again and it resumes.
// Samples reached least often come first in each list, so a long chain
// cannot starve new requests and no request waits behind another's launch.
// A queued sample too large for the free arena space is passed over by
// later ones that fit.
// Two launches stay in flight; the host retires the older one, frees the
// slabs of samples that finished, admits more, and enqueues the next.
#include <deque>

#include "arena.h"
#include "rsa_runtime.h"

namespace rsa {
namespace {

constexpr int kStreams = 4;          // group launches fork onto these
constexpr int kDepth = 2;            // launches in flight
constexpr uint32_t kDefaultQuantumUs = 2000;
constexpr uint32_t kDefaultResident = 4096;
constexpr uint32_t kQueueWords = 128;  // one counter per kernel group (at most 80 groups)
constexpr size_t kLookahead = 256;     // queued samples scanned past one that does not fit

struct Sample {
    uint64_t req = 0;
    uint32_t idx = 0;         // position in its request
    rsa_sample_t s{};
    int tile = 0;
    int key = 0;              // kernel group (group_key)
    uint64_t off = 0, bytes = 0;
    bool resident = false;    // holds arena space
    bool listed = false;      // appeared in a launch (its state record exists)
    bool done = false;        // final result seen
    uint64_t last_launch = 0; // sequence number of the last launch listing it
    uint32_t runs = 0;        // launches in which a workgroup reached it
    uint64_t progress = 0;    // deposits made, as of the last retired launch
};

struct Request {
    uint32_t n = 0, n_done = 0;
    std::vector<rsa_result_t> res;
};

struct Launch {
    uint64_t seq = 0;
    int buf = 0;
    std::vector<uint64_t> entries;   // sample handles, in descriptor order
};

struct Buffers {
    DevDesc *h_desc = nullptr;       // pinned
    rsa_result_t *h_res = nullptr;   // pinned
    DevDesc *d_desc = nullptr;
    DevResult *d_res = nullptr;
    uint32_t *d_queue = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
};

}  // namespace
}  // namespace rsa

using namespace rsa;

struct rsa_server {
    rsa_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t streams[kStreams] = {};
    hipEvent_t fork = nullptr, join[kStreams] = {};
    uint64_t quantum_ticks = 0;
    uint32_t max_resident = 0;
    Block mem;                    // arena + launch buffers
    uint8_t *arena_base = nullptr;
    Arena arena;
    Buffers bufs[kDepth];
    std::deque<Launch> inflight;
    uint64_t next_seq = 1, next_req = 1, next_sample = 1;
    std::map<uint64_t, Sample> samples;      // handle -> sample (handles grow with submission)
    std::deque<uint64_t> queue;              // handles not yet admitted
    std::map<uint64_t, Request> requests;    // id -> request (until collected)
    std::deque<uint64_t> completed;          // ids not yet reported
    uint64_t n_resident = 0;
    rsa_server_stats_t st{};
};

namespace {

uint32_t lds_bytes(const rsa_ctx *c, const rsa_sample_t &s, int tile) { return sample_lds(s.L, s.k, tile, interval_lds_max(c)); }

// Kernel group of a sample: (waves, rows wider than 64 words, sparse clear,
// contact census) select the kernel; the last bit splits lattices up to
// L = 1024 from larger ones, whose row counts take more LDS and so fewer
// workgroups per CU.
int group_key(const rsa_sample_t &s, int tile)
{
    const int kernel = kernel_key(tile_waves(tile), s.L > 4096 ? 1 : 0, tile_sparse(tile),
                                  (s.flags & RSA_FLAG_CONTACTS) ? 1 : 0);
    return kernel * 2 + (s.L > 1024 ? 1 : 0);
}

// Record a finished launch: progress of every sample it reached, final
// results, and the slabs no later launch refers to.
void retire(rsa_server *v, const Launch &l)
{
    Buffers &b = v->bufs[l.buf];
    for (size_t i = 0; i < l.entries.size(); ++i) {
        auto it = v->samples.find(l.entries[i]);
        if (it == v->samples.end()) continue;
        Sample &sm = it->second;
        const rsa_result_t &r = b.h_res[i];
        if (r.status == kStatusNotRun) continue;
        ++sm.runs;
        if (sm.done) continue;
        if (r.status == kStatusYielded) {
            const uint64_t p = r.n_jam > 0 ? (uint64_t)r.n_jam : 0;
            v->st.deposits_in_progress += p - sm.progress;
            sm.progress = p;
            continue;
        }
        v->st.deposits_in_progress -= sm.progress;
        sm.progress = 0;
        sm.done = true;
        Request &q = v->requests[sm.req];
        q.res[sm.idx] = r;
        ++q.n_done;
        ++v->st.samples_completed;
        if (r.n_jam > 0) v->st.deposits_completed += (uint64_t)r.n_jam;
        if (q.n_done == q.n) {
            ++v->st.requests_completed;
            v->completed.push_back(sm.req);
        }
    }
    // free the slabs of finished samples this launch was the last to list
    for (uint64_t h : l.entries) {
        auto it = v->samples.find(h);
        if (it == v->samples.end()) continue;
        Sample &sm = it->second;
        if (sm.done && sm.last_launch == l.seq) {
            v->arena.release(sm.off, sm.bytes);
            --v->n_resident;
            v->samples.erase(it);
        }
    }
    b.busy = false;
}

// Retire finished launches in order; with block, wait for the oldest first.
int retire_ready(rsa_server *v, bool block)
{
    while (!v->inflight.empty()) {
        Launch &l = v->inflight.front();
        hipEvent_t ev = v->bufs[l.buf].done;
        hipError_t e = block ? hipEventSynchronize(ev) : hipEventQuery(ev);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) return hip_fail(v->ctx, e, "server launch");
        retire(v, l);
        v->inflight.pop_front();
        block = false;
    }
    return RSA_OK;
}

// Admit queued samples in submission order while a slot and arena space are
// free.  A sample that does not fit stays queued, and later samples that do
// fit are admitted past it (looking at most kLookahead entries ahead).
void admit(rsa_server *v)
{
    size_t i = 0, skipped = 0;
    while (i < v->queue.size() && v->n_resident < v->max_resident && skipped < kLookahead) {
        Sample &sm = v->samples[v->queue[i]];
        uint64_t off = 0;
        if (!v->arena.alloc(sm.bytes, off)) {
            ++i;
            ++skipped;
            continue;
        }
        sm.off = off;
        sm.resident = true;
        ++v->n_resident;
        v->queue.erase(v->queue.begin() + (std::ptrdiff_t)i);
    }
    v->st.arena_used = v->arena.used();
    v->st.arena_peak = v->arena.peak();
}

// Enqueue one time-sliced launch over every resident sample not known to be
// finished.  Returns RSA_OK, or 1 if there is nothing to run.
int launch(rsa_server *v)
{
    rsa_ctx *c = v->ctx;
    int bi = -1;
    for (int i = 0; i < kDepth; ++i)
        if (!v->bufs[i].busy) {
            bi = i;
            break;
        }
    if (bi < 0) return 1;
    std::vector<uint64_t> live;
    for (auto &kv : v->samples)
        if (kv.second.resident && !kv.second.done) live.push_back(kv.first);
    if (live.empty()) return 1;
    // group-major; inside a group, samples reached least often first
    std::stable_sort(live.begin(), live.end(), [&](uint64_t a, uint64_t b) {
        const Sample &x = v->samples[a], &y = v->samples[b];
        if (x.key != y.key) return x.key > y.key;
        return x.runs < y.runs;
    });
    Buffers &b = v->bufs[bi];
    Launch l;
    l.seq = v->next_seq++;
    l.buf = bi;
    l.entries = live;
    const uint32_t n = (uint32_t)live.size();
    for (uint32_t i = 0; i < n; ++i) {
        Sample &sm = v->samples[live[i]];
        DevDesc d = make_dev_desc(sm.s, i, sm.tile, interval_lds_max(c));
        d.slab = (uint64_t)(uintptr_t)(v->arena_base + sm.off);
        if (!sm.listed) d.flags |= kDescFresh;
        sm.listed = true;
        sm.last_launch = l.seq;
        b.h_desc[i] = d;
    }
    // groups and their grids: every group gets workgroups for all of its
    // samples up to what fits on the device, scaled down together when the
    // groups would not all be resident at once
    struct G {
        int kern;   // kernel_key
        uint32_t first, count, lds, cap, grid;
    };
    std::vector<G> gs;
    for (uint32_t i = 0; i < n;) {
        const int key = v->samples[live[i]].key;
        uint32_t j = i, lds = 0;
        while (j < n && v->samples[live[j]].key == key) {
            lds = std::max(lds, lds_bytes(c, v->samples[live[j]].s, v->samples[live[j]].tile));
            ++j;
        }
        const int kern = key >> 1;
        const int waves = kern >> 3, wide = (kern >> 2) & 1, sparse = (kern >> 1) & 1, census = kern & 1;
        uint32_t cap = (uint32_t)resident_blocks(c, waves, wide, sparse, census, lds);
        gs.push_back(G{kern, i, j - i, lds, cap, 0});
        i = j;
    }
    // group g runs on stream g % kStreams: groups gi .. gi + kStreams - 1 run
    // side by side and share the device
    for (size_t r0 = 0; r0 < gs.size(); r0 += kStreams) {
        const size_t r1 = std::min(gs.size(), r0 + kStreams);
        double load = 0;
        for (size_t gi = r0; gi < r1; ++gi) load += (double)std::min(gs[gi].count, gs[gi].cap) / gs[gi].cap;
        for (size_t gi = r0; gi < r1; ++gi) {
            uint32_t want = std::min(gs[gi].count, gs[gi].cap);
            if (load > 1.0) want = (uint32_t)((double)want / load);
            gs[gi].grid = std::max<uint32_t>(1, want);
        }
    }
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(b.d_desc, b.h_desc, (size_t)n * sizeof(DevDesc), hipMemcpyHostToDevice,
                              v->stream));
    {
        uint32_t nq = kQueueWords;
        uint32_t grid = (std::max(n, nq) + 255) / 256;
        void *pargs[] = {&b.d_desc, (void *)&n, &b.d_res, &b.d_queue, &nq};
        HIP_TRY(c, hipLaunchKernel(kPrepareKernel, dim3(grid), dim3(256), pargs, 0, v->stream));
    }
    HIP_TRY(c, hipEventRecord(v->fork, v->stream));
    for (int s = 0; s < kStreams; ++s) HIP_TRY(c, hipStreamWaitEvent(v->streams[s], v->fork, 0));
    for (size_t gi = 0; gi < gs.size(); ++gi) {
        const G &g = gs[gi];
        const int waves = g.kern >> 3, wide = (g.kern >> 2) & 1, sparse = (g.kern >> 1) & 1,
                  census = g.kern & 1;
        KernelArgs a{};
        a.descs = b.d_desc + g.first;
        a.n = g.count;
        a.tile = (uint32_t)waves;
        a.queue = b.d_queue + gi;
        a.slabs = nullptr;
        a.slab_stride = 0;
        a.results = b.d_res;
        a.prof = nullptr;
        a.quantum = v->quantum_ticks;
        void *kargs[] = {&a};
        HIP_TRY(c, hipLaunchKernel(persistent_kernel(waves, wide, sparse, census), dim3(g.grid),
                                   dim3(64 * (kTileWaves[waves] + 1)), kargs, g.lds,
                                   v->streams[gi % kStreams]));
    }
    for (int s = 0; s < kStreams; ++s) {
        HIP_TRY(c, hipEventRecord(v->join[s], v->streams[s]));
        HIP_TRY(c, hipStreamWaitEvent(v->stream, v->join[s], 0));
    }
    HIP_TRY(c, hipMemcpyAsync(b.h_res, b.d_res, (size_t)n * sizeof(DevResult), hipMemcpyDeviceToHost,
                              v->stream));
    HIP_TRY(c, hipEventRecord(b.done, v->stream));
    b.busy = true;
    v->inflight.push_back(std::move(l));
    ++v->st.launches;
    return RSA_OK;
}

void free_server(rsa_server *v)
{
    if (!v) return;
    for (int i = 0; i < kDepth; ++i) {
        if (v->bufs[i].done) (void)hipEventDestroy(v->bufs[i].done);
        if (v->bufs[i].h_desc) (void)hipHostFree(v->bufs[i].h_desc);
        if (v->bufs[i].h_res) (void)hipHostFree(v->bufs[i].h_res);
    }
    for (int s = 0; s < kStreams; ++s) {
        if (v->streams[s]) (void)hipStreamDestroy(v->streams[s]);
        if (v->join[s]) (void)hipEventDestroy(v->join[s]);
    }
    if (v->fork) (void)hipEventDestroy(v->fork);
    if (v->mem.ptr) give_block(v->ctx, v->mem);
    delete v;
}

}  // namespace

extern "C" {

int rsa_server_create(rsa_ctx *c, const rsa_server_config_t *cfg, void *hip_stream, rsa_server **out)
{
    if (!c || !out) return RSA_EINVAL;
    *out = nullptr;
    if (c->poisoned) return fail(c, RSA_EDEVICE, "context poisoned by an earlier device error");
    HIP_TRY(c, hipSetDevice(c->device));
    rsa_server_config_t conf{};
    if (cfg) conf = *cfg;
    std::unique_ptr<rsa_server> v(new (std::nothrow) rsa_server());
    if (!v) return RSA_ENOMEM;
    v->ctx = c;
    v->stream = (hipStream_t)hip_stream;
    v->max_resident = conf.max_resident ? conf.max_resident : kDefaultResident;
    const uint64_t q_us = conf.quantum_us ? conf.quantum_us : kDefaultQuantumUs;
    const uint64_t khz = c->clock_khz > 0 ? (uint64_t)c->clock_khz : 100000;
    v->quantum_ticks = std::max<uint64_t>(1, q_us * khz / 1000);
    uint64_t arena = conf.arena_bytes ? conf.arena_bytes : c->budget / 2;
    arena = arena / Arena::kAlign * Arena::kAlign;
    const size_t nmax = v->max_resident;
    const size_t desc_b = align256(nmax * sizeof(DevDesc));
    const size_t res_b = align256(nmax * sizeof(DevResult));
    const size_t q_b = align256(kQueueWords * 4);
    const size_t per = desc_b + res_b + q_b;
    if (arena == 0 || !take_block(c, arena + kDepth * per, v->mem))
        return fail(c, RSA_ENOMEM, "server arena does not fit the device memory budget");
    v->arena_base = (uint8_t *)v->mem.ptr;
    v->arena.reset(arena);
    for (int i = 0; i < kDepth; ++i) {
        uint8_t *p = v->arena_base + arena + i * per;
        Buffers &b = v->bufs[i];
        b.d_desc = (DevDesc *)p;
        b.d_res = (DevResult *)(p + desc_b);
        b.d_queue = (uint32_t *)(p + desc_b + res_b);
        if (hipHostMalloc((void **)&b.h_desc, desc_b, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&b.h_res, res_b, hipHostMallocDefault) != hipSuccess) {
            free_server(v.release());
            return fail(c, RSA_ENOMEM, "pinned host allocation failed");
        }
        if (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess) {
            free_server(v.release());
            return fail(c, RSA_EDEVICE, "hipEventCreate failed");
        }
    }
    for (int s = 0; s < kStreams; ++s) {
        if (hipStreamCreateWithFlags(&v->streams[s], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&v->join[s], hipEventDisableTiming) != hipSuccess) {
            free_server(v.release());
            return fail(c, RSA_EDEVICE, "stream creation failed");
        }
    }
    if (hipEventCreateWithFlags(&v->fork, hipEventDisableTiming) != hipSuccess) {
        free_server(v.release());
        return fail(c, RSA_EDEVICE, "hipEventCreate failed");
    }
    v->st.arena_bytes = v->arena.size();
    *out = v.release();
    return RSA_OK;
}

int rsa_server_submit(rsa_server *v, const rsa_sample_t *s, uint32_t n, uint64_t *request_id)
{
    if (!v || !request_id || !s || n == 0) return v ? fail(v->ctx, RSA_EINVAL, "empty request") : RSA_EINVAL;
    rsa_ctx *c = v->ctx;
    for (uint32_t i = 0; i < n; ++i) {
        if (!valid_sample(s[i]))
            return fail(c, RSA_EINVAL, "invalid descriptor at index " + std::to_string(i));
        if (s[i].flags & RSA_FLAG_CLUSTER_SIZES)
            return fail(c, RSA_EINVAL, "cluster sizes are a batch feature (rsa_batch_cluster_sizes)");
        if (lds_layout(s[i].L).total + 64 > c->lds_max) return fail(c, RSA_EINVAL, "lattice too large for LDS");
        if (Arena::round(sample_slab(s[i].L, s[i].k, sample_tile(c, s[i].L, s[i].k))) > v->arena.size())
            return fail(c, RSA_ENOMEM, "sample larger than the server arena");
    }
    const uint64_t id = v->next_req++;
    Request &q = v->requests[id];
    q.n = n;
    q.res.assign(n, rsa_result_t{});
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t h = v->next_sample++;
        Sample &sm = v->samples[h];
        sm.req = id;
        sm.idx = i;
        sm.s = s[i];
        sm.tile = sample_tile(c, s[i].L, s[i].k);
        sm.key = group_key(s[i], sm.tile);
        sm.bytes = sample_slab(s[i].L, s[i].k, sm.tile);
        v->queue.push_back(h);
    }
    ++v->st.requests_submitted;
    *request_id = id;
    return RSA_OK;
}

int rsa_server_step(rsa_server *v, int wait)
{
    if (!v) return RSA_EINVAL;
    rsa_ctx *c = v->ctx;
    if (c->poisoned) return fail(c, RSA_EDEVICE, "context poisoned by an earlier device error");
    const uint64_t before = v->st.requests_completed;
    int rc = retire_ready(v, false);
    if (rc < 0) return rc;
    if (wait && v->st.requests_completed == before && !v->inflight.empty()) {
        rc = retire_ready(v, true);
        if (rc < 0) return rc;
    }
    admit(v);
    while ((int)v->inflight.size() < kDepth) {
        rc = launch(v);
        if (rc < 0) return rc;
        if (rc > 0) break;
    }
    return (int)(v->st.requests_completed - before);
}

int rsa_server_completed(rsa_server *v, uint64_t *ids, uint32_t cap)
{
    if (!v || (cap > 0 && !ids)) return RSA_EINVAL;
    uint32_t k = 0;
    while (k < cap && !v->completed.empty()) {
        ids[k++] = v->completed.front();
        v->completed.pop_front();
    }
    return (int)k;
}

int rsa_server_results(rsa_server *v, uint64_t request_id, rsa_result_t *out, uint32_t n)
{
    if (!v) return RSA_EINVAL;
    auto it = v->requests.find(request_id);
    if (it == v->requests.end()) return fail(v->ctx, RSA_ENOTFOUND, "unknown request id");
    Request &q = it->second;
    if (n != q.n || !out) return fail(v->ctx, RSA_EINVAL, "result count differs from request size");
    if (q.n_done < q.n) return RSA_ENOTREADY;
    std::memcpy(out, q.res.data(), (size_t)n * sizeof(rsa_result_t));
    v->requests.erase(it);
    return RSA_OK;
}

int rsa_server_stats(rsa_server *v, rsa_server_stats_t *out)
{
    if (!v || !out) return RSA_EINVAL;
    v->st.samples_queued = v->queue.size();
    v->st.samples_resident = v->n_resident;
    v->st.arena_used = v->arena.used();
    v->st.arena_peak = v->arena.peak();
    *out = v->st;
    return RSA_OK;
}

void rsa_server_destroy(rsa_server *v)
{
    if (!v) return;
    (void)hipSetDevice(v->ctx->device);
    for (auto &l : v->inflight) (void)hipEventSynchronize(v->bufs[l.buf].done);
    v->inflight.clear();
    free_server(v);
}

}  // extern "C"
