// Batched explicit stepping of many operators of uneven sizes.
//
// Problems are grouped by class (dim, offset width, boundary, storage); one
// grouped launch advances every problem of a class by one step (blocks laid
// out problem after problem, each block finds its problem by binary search
// over a small device descriptor table).  The problems are independent, so
// a class may also be cut into chunks whose working sets fit the 256 MB
// last-level (Infinity) cache, each chunk taking all its steps before the
// next starts: after the first step a chunk's arrays are served from that
// cache instead of HBM.  nsteps of all classes are captured once into a HIP
// graph on the batch's own stream and replayed, so a whole run is one graph
// launch.  The autotuner times the launch variants of each class on the
// batch itself (without touching the state: it steps u into u_tmp) and
// keeps the fastest, also in a per-process cache keyed by the class and its
// size.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <new>
#include <vector>
#include <cerrno>

#include "common.h"

struct adlbr_batch {
    struct Class {
        int key;
        const adlbr_operator *rep;
        std::vector<adlbr::BatchProb> host;  // descriptors in problem order
        std::vector<adlbr::BatchProb> order;  // descriptors as uploaded (variant's order)
        std::vector<size_t> bytes;           // footprint of each problem, problem order
        adlbr::BatchProb *dev;               // descriptor table in the workspace
        struct Chunk {
            int first, count;  // descriptors [first, first + count) of `order`
            long long nblocks;
        };
        std::vector<Chunk> chunks;           // cache-blocking chunks of `order`
        int variant;
        size_t budget;  // chunk budget in bytes, 0 = the whole class in one chunk
    };
    int nprob;
    std::vector<Class> classes;
    hipStream_t own;
    hipStream_t side;  // the second chain of two chunks in flight (variant bit 3)
    hipEvent_t ev_in, ev_out;
    std::vector<hipEvent_t> forks, joins;  // one pair per two-chunk group
    hipGraph_t graph;
    hipGraphExec_t exec;
    long long graph_steps;
};

namespace adlbr {
namespace {

// bit 0: XCD-contiguous blocks; bit 1: largest problems first; bit 2: one
// launch per problem (in the variant's problem order) instead of one grouped
// launch; bit 3: two chunks in flight, on two streams (parallel branches of
// the graph), so that the tail of one chunk's step overlaps the other's.
// Each is timed with every chunk budget of kChunkMiB (0: no chunks).
constexpr int kVariants = 16;
constexpr size_t kChunkMiB[4] = {0, 64, 128, 224};

std::mutex g_cache_mu;
// (class, log2 points, problems) -> (variant, chunk budget)
std::map<long long, std::pair<int, size_t>> g_cache;

int log2_floor(long long pts) {
    int lg = 0;
    while (lg < 62 && (1ll << (lg + 1)) <= pts) ++lg;
    return lg;
}
long long make_key(int cls, int lg, long long nprob) {
    return ((long long)cls * 64 + lg) * 4096 + std::min<long long>(nprob, 4095);
}
long long cache_key(const adlbr_batch::Class &c) {
    long long pts = 0;
    for (const BatchProb &p : c.host) pts += p.g.N;
    return make_key(c.key, log2_floor(pts), (long long)c.host.size());
}

// The integer after "name": in [b, e), false if absent or not a number.
bool json_int(const std::string &t, size_t b, size_t e, const char *name, long long *out) {
    const std::string k = std::string("\"") + name + "\"";
    const size_t at = t.find(k, b);
    if (at == std::string::npos || at >= e) return false;
    size_t i = t.find(':', at + k.size());
    if (i == std::string::npos || i >= e) return false;
    ++i;
    while (i < e && (t[i] == ' ' || t[i] == '\t' || t[i] == '\n' || t[i] == '\r')) ++i;
    char *end = nullptr;
    errno = 0;
    const long long v = std::strtoll(t.c_str() + i, &end, 10);
    if (errno || end == t.c_str() + i || (size_t)(end - t.c_str()) > e) return false;
    *out = v;
    return true;
}

// Lay out the class's problems in the order of the variant, cut them into
// chunks within the variant's budget (at least one problem each; block
// numbers restart at 0 in every chunk) and upload.
int upload(adlbr_batch::Class &c, int variant, size_t budget, hipStream_t s) {
    std::vector<int> idx(c.host.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    if (variant & 2)
        std::stable_sort(idx.begin(), idx.end(),
                         [&](int a, int b) { return c.host[a].g.N > c.host[b].g.N; });
    std::vector<BatchProb> d;
    c.chunks.clear();
    size_t used = 0;
    long long fb = 0;
    for (int i : idx) {
        const bool fits = budget == 0 || used + c.bytes[i] <= budget;
        if (c.chunks.empty() || !fits) {
            c.chunks.push_back({(int)d.size(), 0, 0});
            used = 0;
            fb = 0;
        }
        BatchProb p = c.host[i];
        p.first_block = fb;
        fb += p.nblocks;
        used += c.bytes[i];
        d.push_back(p);
        c.chunks.back().count++;
        c.chunks.back().nblocks = fb;
    }
    c.order = d;
    ADLBR_CHECK_HIP(hipMemcpyAsync(c.dev, c.order.data(), d.size() * sizeof(BatchProb),
                                   hipMemcpyHostToDevice, s));
    ADLBR_CHECK_HIP(hipStreamSynchronize(s));
    c.variant = variant;
    c.budget = budget;
    return ADLBR_OK;
}

int launch_chunk(const adlbr_batch::Class &c, const adlbr_batch::Class::Chunk &k, int parity,
                 int variant, int copy, hipStream_t s) {
    return batch_launch(c.rep, c.dev + k.first, c.order.data() + k.first, k.count, k.nblocks,
                        parity, variant, copy, s);
}

// Every step of one chunk (u -> u_tmp -> u ...) and the copy back into u
// after an odd count; with run = false (the tuner's timing) parity 0 only:
// u is read and u_tmp written, nsteps times.
int chunk_steps(const adlbr_batch::Class &c, const adlbr_batch::Class::Chunk &k, long long nsteps,
                bool run, hipStream_t s) {
    for (long long t = 0; t < nsteps; ++t) {
        int rc = launch_chunk(c, k, run ? (int)(t & 1) : 0, c.variant, 0, s);
        if (rc) return rc;
    }
    if (run && (nsteps & 1)) return launch_chunk(c, k, 0, c.variant, 1, s);
    return ADLBR_OK;
}

// The chunks of one class, one after another on s; with bit 3, two at a
// time: the second on the batch's side stream, forked from s and joined
// back into it (separate problems, so the two chains share no data).
int class_steps(adlbr_batch *b, const adlbr_batch::Class &c, long long nsteps, bool run,
                hipStream_t s, size_t &group) {
    const size_t nk = c.chunks.size();
    const bool pair = (c.variant & 8) != 0;
    for (size_t i = 0; i < nk; i += pair ? 2 : 1) {
        if (!pair || i + 1 == nk) {
            int rc = chunk_steps(c, c.chunks[i], nsteps, run, s);
            if (rc) return rc;
            continue;
        }
        while (b->forks.size() <= group) {
            hipEvent_t f = nullptr, j = nullptr;
            if (hipEventCreateWithFlags(&f, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess) {
                if (f) (void)hipEventDestroy(f);
                set_error("batch: event creation failed");
                return ADLBR_E_HIP;
            }
            b->forks.push_back(f);
            b->joins.push_back(j);
        }
        const hipEvent_t f = b->forks[group], j = b->joins[group];
        ++group;
        ADLBR_CHECK_HIP(hipEventRecord(f, s));
        ADLBR_CHECK_HIP(hipStreamWaitEvent(b->side, f, 0));
        int rc = chunk_steps(c, c.chunks[i], nsteps, run, s);
        if (!rc) rc = chunk_steps(c, c.chunks[i + 1], nsteps, run, b->side);
        ADLBR_CHECK_HIP(hipEventRecord(j, b->side));
        ADLBR_CHECK_HIP(hipStreamWaitEvent(s, j, 0));
        if (rc) return rc;
    }
    return ADLBR_OK;
}

// Class after class, chunk after chunk (or two at a time), every step.
int enqueue_steps(adlbr_batch *b, long long nsteps, hipStream_t s) {
    size_t group = 0;
    for (auto &c : b->classes) {
        int rc = class_steps(b, c, nsteps, true, s, group);
        if (rc) return rc;
    }
    return ADLBR_OK;
}

void drop_graph(adlbr_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_steps = -1;
}

}  // namespace
}  // namespace adlbr

using namespace adlbr;

extern "C" int adlbr_batch_workspace(int nprob, size_t *bytes) {
    clear_error();
    if (nprob <= 0 || !bytes) {
        set_error("adlbr_batch_workspace: need nprob > 0 and bytes");
        return ADLBR_E_INVALID;
    }
    *bytes = align_up(sizeof(BatchProb) * (size_t)nprob) + 256 * 16;
    return ADLBR_OK;
}

extern "C" int adlbr_batch_create(int nprob, adlbr_operator *const *ops, void *const *u,
                                  void *const *u_tmp, const double *dt, int dt_mode,
                                  void *workspace, size_t ws_bytes, void *stream,
                                  adlbr_batch **out) {
    clear_error();
    if (nprob <= 0 || !ops || !u || !u_tmp || !dt || !workspace || !out) {
        set_error("adlbr_batch_create: null argument or nprob <= 0");
        return ADLBR_E_INVALID;
    }
    if (dt_mode != ADLBR_DT_ABS && dt_mode != ADLBR_DT_CFL) {
        set_error("adlbr_batch_create: dt_mode must be ADLBR_DT_ABS or ADLBR_DT_CFL");
        return ADLBR_E_INVALID;
    }
    size_t need = 0;
    adlbr_batch_workspace(nprob, &need);
    if (ws_bytes < need) {
        set_error("adlbr_batch_create: workspace has %zu bytes, %zu needed", ws_bytes, need);
        return ADLBR_E_NOMEM;
    }
    for (int i = 0; i < nprob; ++i) {
        if (!ops[i] || !u[i] || !u_tmp[i] || u[i] == u_tmp[i] || !(dt[i] >= 0.0)) {
            set_error("adlbr_batch_create: problem %d: null or aliased buffer, or dt < 0", i);
            return ADLBR_E_INVALID;
        }
        int bp = 0;
        if (batch_blocks(ops[i], &bp) >= (1ll << 31)) {
            set_error("adlbr_batch_create: problem %d too large", i);
            return ADLBR_E_RANGE;
        }
    }
    adlbr_batch *b = new (std::nothrow) adlbr_batch;
    if (!b) {
        set_error("adlbr_batch_create: out of host memory");
        return ADLBR_E_NOMEM;
    }
    b->nprob = nprob;
    b->own = b->side = nullptr;
    b->ev_in = b->ev_out = nullptr;
    b->graph = nullptr;
    b->exec = nullptr;
    b->graph_steps = -1;
    std::map<int, int> idx;
    for (int i = 0; i < nprob; ++i) {
        const int key = batch_class(ops[i]);
        auto it = idx.find(key);
        if (it == idx.end()) {
            it = idx.emplace(key, (int)b->classes.size()).first;
            adlbr_batch::Class c;
            c.key = key;
            c.rep = ops[i];
            c.dev = nullptr;
            c.variant = 1;
            c.budget = 0;
            b->classes.push_back(c);
        }
        BatchProb d;
        std::memset(&d, 0, sizeof d);
        batch_describe(ops[i], &d);
        d.u[0] = u[i];
        d.u[1] = u_tmp[i];
        d.dt = dt[i];
        d.dt_mode = dt_mode;
        b->classes[it->second].host.push_back(d);
        b->classes[it->second].bytes.push_back(batch_footprint(ops[i]));
    }
    long long total_blocks = 0;
    char *base = (char *)workspace;
    size_t o = 0;
    for (auto &c : b->classes) {
        c.dev = (BatchProb *)(base + o);
        o += sizeof(BatchProb) * c.host.size();
        for (const BatchProb &p : c.host) total_blocks += p.nblocks;
    }
    if (total_blocks >= (1ll << 31)) {
        delete b;
        set_error("adlbr_batch_create: too many points in one batch");
        return ADLBR_E_RANGE;
    }
    hipStream_t s = as_stream(stream);
    int rc = ADLBR_OK;
    for (auto &c : b->classes) {
        std::pair<int, size_t> v(1, 0);
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_cache.find(cache_key(c));
            if (it != g_cache.end()) v = it->second;
        }
        rc = upload(c, v.first, v.second, s);
        if (rc) break;
    }
    if (!rc && (hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess ||
                hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess)) {
        set_error("adlbr_batch_create: stream or event creation failed");
        rc = ADLBR_E_HIP;
    }
    if (rc) {
        if (b->ev_in) (void)hipEventDestroy(b->ev_in);
        if (b->ev_out) (void)hipEventDestroy(b->ev_out);
        if (b->own) (void)hipStreamDestroy(b->own);
        if (b->side) (void)hipStreamDestroy(b->side);
        delete b;
        return rc;
    }
    *out = b;
    return ADLBR_OK;
}

extern "C" int adlbr_batch_tune(adlbr_batch *b, int steps, int use_cache, void *stream) {
    clear_error();
    if (!b || steps <= 0) {
        set_error("adlbr_batch_tune: null batch or steps <= 0");
        return ADLBR_E_INVALID;
    }
    hipStream_t s = as_stream(stream);
    EventPair ev;
    ADLBR_CHECK_HIP(ev.create());
    const hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
    int rc = ADLBR_OK;
    for (auto &c : b->classes) {
        const long long key = cache_key(c);
        if (use_cache) {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_cache.find(key);
            if (it != g_cache.end()) {
                rc = upload(c, it->second.first, it->second.second, s);
                if (rc) break;
                continue;
            }
        }
        int best = -1;
        size_t best_budget = 0;
        float best_ms = 0.f;
        size_t class_bytes = 0;
        for (size_t b2 : c.bytes) class_bytes += b2;
        for (int cand = 0; cand < 4 * kVariants && !rc; ++cand) {
            const int v = cand % kVariants;
            const size_t budget = kChunkMiB[cand / kVariants] << 20;
            if ((v & 4) && (v & 1)) continue;  // bit 0 has no meaning without a grouped launch
            // a budget that holds the whole class is the same as no chunking
            if (budget && class_bytes <= budget) continue;
            if ((v & 8) && !budget) continue;  // one chunk: nothing to pair
            rc = upload(c, v, budget, s);
            if (rc) break;
            // warm-up over all chunks, then `steps` steps of every chunk as a
            // run takes them (bit 3: two chunks at a time); parity 0 only:
            // u is read, u_tmp written
            for (const auto &k : c.chunks)
                if (!rc) rc = launch_chunk(c, k, 0, v, 0, s);
            if (rc) break;
            size_t group = 0;
            ADLBR_CHECK_HIP(hipEventRecord(e0, s));
            rc = class_steps(b, c, steps, false, s, group);
            ADLBR_CHECK_HIP(hipEventRecord(e1, s));
            ADLBR_CHECK_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            ADLBR_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (best < 0 || ms < best_ms) {
                best = v;
                best_budget = budget;
                best_ms = ms;
            }
        }
        if (rc) break;
        rc = upload(c, best, best_budget, s);
        if (rc) break;
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_cache[key] = std::make_pair(best, best_budget);
    }
    drop_graph(b);  // the variants are baked into a captured graph
    if (!rc) ADLBR_LAUNCH_CHECK();
    return rc;
}

extern "C" int adlbr_batch_set_variant(adlbr_batch *b, int cls, int variant, size_t chunk_bytes,
                                       void *stream) {
    clear_error();
    if (!b || cls < 0 || cls >= (int)b->classes.size() || variant < 0 || variant >= kVariants) {
        set_error("adlbr_batch_set_variant: bad class or variant");
        return ADLBR_E_INVALID;
    }
    int rc = upload(b->classes[cls], variant, chunk_bytes, as_stream(stream));
    drop_graph(b);
    return rc;
}

extern "C" int adlbr_batch_variant(const adlbr_batch *b, int cls, int *key, int *variant,
                                   int *nprob, int *nchunks, size_t *chunk_bytes) {
    clear_error();
    if (!b || cls < 0 || cls >= (int)b->classes.size() || !key || !variant || !nprob) {
        set_error("adlbr_batch_variant: bad argument");
        return ADLBR_E_INVALID;
    }
    const adlbr_batch::Class &c = b->classes[cls];
    *key = c.key;
    *variant = c.variant;
    *nprob = (int)c.host.size();
    if (nchunks) *nchunks = (int)c.chunks.size();
    if (chunk_bytes) *chunk_bytes = c.budget;
    return ADLBR_OK;
}

extern "C" int adlbr_batch_run(adlbr_batch *b, int64_t nsteps, int use_graph, void *stream) {
    clear_error();
    if (!b || nsteps < 0) {
        set_error("adlbr_batch_run: null batch or nsteps < 0");
        return ADLBR_E_INVALID;
    }
    if (nsteps == 0) return ADLBR_OK;
    hipStream_t s = as_stream(stream);
    if (!use_graph) {
        int rc = enqueue_steps(b, nsteps, s);
        if (rc) return rc;
        ADLBR_LAUNCH_CHECK();
        return ADLBR_OK;
    }
    if (!b->exec || b->graph_steps != nsteps) {
        drop_graph(b);
        ADLBR_CHECK_HIP(hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_steps(b, nsteps, b->own);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(b->own, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (ec != hipSuccess || !g) {
            set_error("adlbr_batch_run: graph capture failed: %s", hipGetErrorString(ec));
            return ADLBR_E_HIP;
        }
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(b);
            set_error("adlbr_batch_run: graph instantiation failed");
            return ADLBR_E_HIP;
        }
        b->graph_steps = nsteps;
    }
    // run the graph on the batch's stream, ordered after and before `stream`
    ADLBR_CHECK_HIP(hipEventRecord(b->ev_in, s));
    ADLBR_CHECK_HIP(hipStreamWaitEvent(b->own, b->ev_in, 0));
    ADLBR_CHECK_HIP(hipGraphLaunch(b->exec, b->own));
    ADLBR_CHECK_HIP(hipEventRecord(b->ev_out, b->own));
    ADLBR_CHECK_HIP(hipStreamWaitEvent(s, b->ev_out, 0));
    return ADLBR_OK;
}

extern "C" int adlbr_batch_destroy(adlbr_batch *b) {
    if (!b) return ADLBR_OK;
    if (b->own) (void)hipStreamSynchronize(b->own);
    if (b->side) (void)hipStreamSynchronize(b->side);
    drop_graph(b);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    for (hipEvent_t e : b->forks) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->joins) (void)hipEventDestroy(e);
    if (b->own) (void)hipStreamDestroy(b->own);
    if (b->side) (void)hipStreamDestroy(b->side);
    delete b;
    return ADLBR_OK;
}

// ------------------------------------------------ the tuner's file cache --
extern "C" int adlbr_batch_tune_save(const char *path) {
    clear_error();
    if (!path) {
        set_error("adlbr_batch_tune_save: null path");
        return ADLBR_E_INVALID;
    }
    std::map<long long, std::pair<int, size_t>> snap;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        snap = g_cache;
    }
    FILE *f = std::fopen(path, "w");
    if (!f) {
        set_error("adlbr_batch_tune_save: cannot open %s for writing", path);
        return ADLBR_E_INVALID;
    }
    std::fprintf(f, "{\"format\": \"adlbr-batch-tune\", \"version\": 1, \"entries\": [");
    bool first = true;
    for (const auto &kv : snap) {
        const long long key = kv.first;
        const long long np = key % 4096, lg = (key / 4096) % 64, cls = key / (4096 * 64);
        std::fprintf(f, "%s\n  {\"class\": %lld, \"log2_points\": %lld, \"problems\": %lld, "
                        "\"variant\": %d, \"chunk_bytes\": %zu}",
                     first ? "" : ",", cls, lg, np, kv.second.first, kv.second.second);
        first = false;
    }
    std::fprintf(f, "\n]}\n");
    const bool bad = std::ferror(f) != 0;
    if (std::fclose(f) != 0 || bad) {
        set_error("adlbr_batch_tune_save: write to %s failed", path);
        return ADLBR_E_INVALID;
    }
    return ADLBR_OK;
}

extern "C" int adlbr_batch_tune_load(const char *path) {
    clear_error();
    if (!path) {
        set_error("adlbr_batch_tune_load: null path");
        return ADLBR_E_INVALID;
    }
    FILE *f = std::fopen(path, "r");
    if (!f) {
        set_error("adlbr_batch_tune_load: cannot open %s", path);
        return ADLBR_E_INVALID;
    }
    std::string t;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) t.append(buf, n);
    std::fclose(f);
    if (t.find("\"adlbr-batch-tune\"") == std::string::npos) {
        set_error("adlbr_batch_tune_load: %s is not a tuner cache", path);
        return ADLBR_E_INVALID;
    }
    size_t pos = t.find("\"entries\"");
    if (pos == std::string::npos || (pos = t.find('[', pos)) == std::string::npos) {
        set_error("adlbr_batch_tune_load: %s has no entries list", path);
        return ADLBR_E_INVALID;
    }
    const size_t close = t.find(']', pos);
    if (close == std::string::npos) {
        set_error("adlbr_batch_tune_load: %s: unterminated entries list", path);
        return ADLBR_E_INVALID;
    }
    // parse every entry first; the cache changes only if all are valid
    std::vector<std::pair<long long, std::pair<int, size_t>>> got;
    size_t b = pos;
    while ((b = t.find('{', b)) != std::string::npos && b < close) {
        const size_t e = t.find('}', b);
        if (e == std::string::npos || e > close) {
            set_error("adlbr_batch_tune_load: %s: unterminated entry", path);
            return ADLBR_E_INVALID;
        }
        long long cls, lg, np, var, cb;
        if (!json_int(t, b, e, "class", &cls) || !json_int(t, b, e, "log2_points", &lg) ||
            !json_int(t, b, e, "problems", &np) || !json_int(t, b, e, "variant", &var) ||
            !json_int(t, b, e, "chunk_bytes", &cb) || cls < 0 || cls > (1ll << 30) || lg < 0 ||
            lg > 62 || np < 1 || np > 4095 || var < 0 || var >= kVariants || cb < 0) {
            set_error("adlbr_batch_tune_load: %s: malformed entry at byte %zu", path, b);
            return ADLBR_E_INVALID;
        }
        got.push_back({make_key((int)cls, (int)lg, np), {(int)var, (size_t)cb}});
        b = e + 1;
    }
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (const auto &kv : got) g_cache[kv.first] = kv.second;
    return ADLBR_OK;
}

extern "C" int adlbr_batch_tune_clear(void) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache.clear();
    return ADLBR_OK;
}

extern "C" int adlbr_batch_tune_lookup(int class_key, int64_t points, int nprob, int *found,
                                       int *variant, size_t *chunk_bytes) {
    clear_error();
    if (class_key < 0 || points < 1 || nprob < 1 || !found) {
        set_error("adlbr_batch_tune_lookup: bad argument");
        return ADLBR_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_cache_mu);
    const auto it = g_cache.find(make_key(class_key, log2_floor(points), nprob));
    *found = it != g_cache.end();
    if (*found) {
        if (variant) *variant = it->second.first;
        if (chunk_bytes) *chunk_bytes = it->second.second;
    }
    return ADLBR_OK;
}
