// Batched explicit stepping of many operators of uneven sizes.
//
// Problems are grouped by class (dim, offset width, boundary, storage); one
// grouped launch advances every problem of a class by one step (blocks laid
// out problem after problem, each block finds its problem by binary search
// over a small device descriptor table).  nsteps of all classes are captured
// once into a HIP graph on the batch's own stream and replayed, so a whole
// run is one graph launch.  The autotuner times the launch variants of each
// class on the batch itself (without touching the state: it steps u into
// u_tmp) and keeps the fastest, also in a per-process cache keyed by the
// class and its size.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "common.h"

struct adlbr_batch {
    struct Class {
        int key;
        const adlbr_operator *rep;
        std::vector<adlbr::BatchProb> host;  // descriptors in problem order
        adlbr::BatchProb *dev;               // descriptor table in the workspace
        long long nblocks;
        int variant;
    };
    int nprob;
    std::vector<Class> classes;
    hipStream_t own;
    hipEvent_t ev_in, ev_out;
    hipGraph_t graph;
    hipGraphExec_t exec;
    long long graph_steps;
};

namespace adlbr {
namespace {

constexpr int kVariants = 4;  // bit 0: XCD-contiguous blocks; bit 1: largest problems first

std::mutex g_cache_mu;
std::map<long long, int> g_cache;  // (class, log2 points, problems) -> variant

long long cache_key(const adlbr_batch::Class &c) {
    long long pts = 0;
    for (const BatchProb &p : c.host) pts += p.g.N;
    int lg = 0;
    while ((1ll << (lg + 1)) <= pts) ++lg;
    return ((long long)c.key * 64 + lg) * 4096 + (long long)std::min<size_t>(c.host.size(), 4095);
}

// Lay out the class's blocks in the order of the variant and upload.
int upload(adlbr_batch::Class &c, int variant, hipStream_t s) {
    std::vector<BatchProb> d = c.host;
    if (variant & 2)
        std::stable_sort(d.begin(), d.end(),
                         [](const BatchProb &a, const BatchProb &b) { return a.g.N > b.g.N; });
    long long fb = 0;
    for (BatchProb &p : d) {
        p.first_block = fb;
        fb += (p.g.N + kApplyPoints - 1) / kApplyPoints;
    }
    c.nblocks = fb;
    ADLBR_CHECK_HIP(hipMemcpyAsync(c.dev, d.data(), d.size() * sizeof(BatchProb),
                                   hipMemcpyHostToDevice, s));
    ADLBR_CHECK_HIP(hipStreamSynchronize(s));  // d must outlive the copy
    c.variant = variant;
    return ADLBR_OK;
}

int enqueue_steps(adlbr_batch *b, long long nsteps, hipStream_t s) {
    for (long long k = 0; k < nsteps; ++k)
        for (auto &c : b->classes) {
            int rc = batch_launch(c.rep, c.dev, (int)c.host.size(), c.nblocks, (int)(k & 1),
                                  c.variant, 0, s);
            if (rc) return rc;
        }
    if (nsteps & 1)
        for (auto &c : b->classes) {
            int rc = batch_launch(c.rep, c.dev, (int)c.host.size(), c.nblocks, 0, c.variant, 1, s);
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
        if ((operator_grid(ops[i]).N + kApplyPoints - 1) / kApplyPoints >= (1ll << 31)) {
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
    b->own = nullptr;
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
            c.nblocks = 0;
            c.variant = 1;
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
    }
    long long total_blocks = 0;
    char *base = (char *)workspace;
    size_t o = 0;
    for (auto &c : b->classes) {
        c.dev = (BatchProb *)(base + o);
        o += sizeof(BatchProb) * c.host.size();
        for (const BatchProb &p : c.host) total_blocks += (p.g.N + kApplyPoints - 1) / kApplyPoints;
    }
    if (total_blocks >= (1ll << 31)) {
        delete b;
        set_error("adlbr_batch_create: too many points in one batch");
        return ADLBR_E_RANGE;
    }
    hipStream_t s = as_stream(stream);
    int rc = ADLBR_OK;
    for (auto &c : b->classes) {
        int v = 1;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_cache.find(cache_key(c));
            if (it != g_cache.end()) v = it->second;
        }
        rc = upload(c, v, s);
        if (rc) break;
    }
    if (!rc && (hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess)) {
        set_error("adlbr_batch_create: stream or event creation failed");
        rc = ADLBR_E_HIP;
    }
    if (rc) {
        if (b->ev_in) (void)hipEventDestroy(b->ev_in);
        if (b->ev_out) (void)hipEventDestroy(b->ev_out);
        if (b->own) (void)hipStreamDestroy(b->own);
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
    hipEvent_t e0, e1;
    ADLBR_CHECK_HIP(hipEventCreate(&e0));
    ADLBR_CHECK_HIP(hipEventCreate(&e1));
    int rc = ADLBR_OK;
    for (auto &c : b->classes) {
        const long long key = cache_key(c);
        if (use_cache) {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_cache.find(key);
            if (it != g_cache.end()) {
                rc = upload(c, it->second, s);
                if (rc) break;
                continue;
            }
        }
        int best = -1;
        float best_ms = 0.f;
        for (int v = 0; v < kVariants && !rc; ++v) {
            rc = upload(c, v, s);
            if (rc) break;
            // warm-up, then timed; parity 0 only: u is read, u_tmp written
            rc = batch_launch(c.rep, c.dev, (int)c.host.size(), c.nblocks, 0, v, 0, s);
            if (rc) break;
            ADLBR_CHECK_HIP(hipEventRecord(e0, s));
            for (int k = 0; k < steps && !rc; ++k)
                rc = batch_launch(c.rep, c.dev, (int)c.host.size(), c.nblocks, 0, v, 0, s);
            ADLBR_CHECK_HIP(hipEventRecord(e1, s));
            ADLBR_CHECK_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            ADLBR_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (best < 0 || ms < best_ms) {
                best = v;
                best_ms = ms;
            }
        }
        if (rc) break;
        rc = upload(c, best, s);
        if (rc) break;
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_cache[key] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graph(b);  // the variants are baked into a captured graph
    if (!rc) ADLBR_LAUNCH_CHECK();
    return rc;
}

extern "C" int adlbr_batch_variant(const adlbr_batch *b, int cls, int *key, int *variant,
                                   int *nprob) {
    clear_error();
    if (!b || cls < 0 || cls >= (int)b->classes.size() || !key || !variant || !nprob) {
        set_error("adlbr_batch_variant: bad argument");
        return ADLBR_E_INVALID;
    }
    *key = b->classes[cls].key;
    *variant = b->classes[cls].variant;
    *nprob = (int)b->classes[cls].host.size();
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
    drop_graph(b);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->own) (void)hipStreamDestroy(b->own);
    delete b;
    return ADLBR_OK;
}
