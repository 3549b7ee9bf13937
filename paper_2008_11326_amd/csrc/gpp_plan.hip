// gpp_plan.hip -- plans for the batched forward: schedule candidates, the
// autotuner with its on-disk cache, the descriptor table and the captured
// hipGraph (entry points declared in include/gpp.h).
//
// A plan fixes the states' sizes.  Candidates differ in the tile variant
// (bands per batch-inverted group), the state order (as given, or
// longest-per-tile first so the last, partial round holds the cheapest
// tiles) and the tile-to-wave schedule (global round-robin, one equal-cost
// contiguous chunk of the tile list per XCD, a work queue of small chunks
// taken from an atomic counter, or one such queue per XCD with stealing).  The persistent grid is sized to the kernel's resident capacity
// on this device.  On the first gpp_sigma_batched call, if no cached choice
// exists, every candidate is timed once on the caller's inputs and the
// fastest is kept and written to the cache (JSON, keyed by architecture,
// kind and a hash of the sizes).  Afterwards each call uploads the
// descriptor table only if an input pointer changed and replays a graph of
// [persistent kernel -> per-state reduction] captured on a private stream.
#include <errno.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gpp.h"
#include "gpp_internal.h"

namespace {

struct Candidate {
    int bu;       // bands per batch-inverted group
    int order;    // 0 = caller order, 1 = longest tiles first
    int sched;    // gpp::BatchedSchedule
    int blocks;   // persistent workgroups (resident capacity); flat: all workgroups
    long nchunks; // work-queue chunks (kSchedQueue); flat: workgroups
};

// Workgroups of the flat form for one state: its tiles of the plain
// forward's shape, four per workgroup.
long flat_workgroups(const gpp::Dims32 &d)
{
    if (!d.nb || !d.ng || !d.np) return 0;
    const int cols = gpp::fwd_cols(d.nw);
    const long tiles = (long)((d.ng + 63) / 64) * ((d.np + cols - 1) / cols);
    return (tiles + 3) / 4;
}

// Tiles per work-queue chunk: small enough that the chunks in flight stay a
// contiguous window of the tile list and the last chunks balance the end.
// The window is (resident waves) x (chunk tiles) consecutive G' columns, and
// each column brings its own aqsmtemp column into L2: 2 keeps it near one
// XCD's L2 at 512 bands (4 measured about 1 % slower, 1 no faster).
#ifndef GPP_QUEUE_CHUNK_TILES
#define GPP_QUEUE_CHUNK_TILES 2
#endif
constexpr int kQueueChunkTiles = GPP_QUEUE_CHUNK_TILES;
// Workspace layout: [0, 256) the queue counters, then the partial rows.
constexpr size_t kPartialsOffset = 256;

struct TuneEntry {
    int bu = 0, order = 0, sched = 0;
    double ms = 0.0;
};

// Relative cost of one tile of a state: its bands plus a fixed per-tile
// part (pair set-up, exchange bands, epilogue) worth about eight bands.
constexpr double kTileOverheadBands = 8.0;

std::mutex g_cache_mu;
std::map<std::string, TuneEntry> g_cache;
bool g_cache_loaded = false;

std::string cache_path()
{
    if (const char *p = getenv("GPP_TUNE_CACHE")) return p;
    std::string base;
    if (const char *x = getenv("XDG_CACHE_HOME")) base = x;
    else if (const char *h = getenv("HOME")) base = std::string(h) + "/.cache";
    else return "";
    return base + "/gpp/tune.json";
}

// Parse {"key": {"bu": 3, "order": 1, "ms": 12.5}, ...}.  Anything that
// does not fit the format empties the result (a corrupt cache is ignored).
bool parse_cache(const std::string &t, std::map<std::string, TuneEntry> &out)
{
    size_t i = 0, n = t.size();
    auto ws = [&] { while (i < n && strchr(" \t\r\n", t[i])) ++i; };
    auto str = [&](std::string &s) {
        ws();
        if (i >= n || t[i] != '"') return false;
        size_t j = t.find('"', i + 1);
        if (j == std::string::npos) return false;
        s = t.substr(i + 1, j - i - 1);
        i = j + 1;
        return true;
    };
    auto ch = [&](char c) { ws(); if (i < n && t[i] == c) { ++i; return true; } return false; };
    if (!ch('{')) return false;
    if (ch('}')) return true;
    do {
        std::string key;
        if (!str(key) || !ch(':') || !ch('{')) return false;
        TuneEntry e;
        bool has_bu = false, has_order = false;
        if (!ch('}')) {
            do {
                std::string f;
                if (!str(f) || !ch(':')) return false;
                ws();
                char *end = nullptr;
                const double v = strtod(t.c_str() + i, &end);
                if (end == t.c_str() + i) return false;
                i = end - t.c_str();
                if (f == "bu") { e.bu = (int)v; has_bu = true; }
                else if (f == "order") { e.order = (int)v; has_order = true; }
                else if (f == "sched") e.sched = (int)v;
                else if (f == "ms") e.ms = v;
            } while (ch(','));
            if (!ch('}')) return false;
        }
        if (!has_bu || !has_order) return false;
        out[key] = e;
    } while (ch(','));
    return ch('}');
}

// The entries of the cache file, or an empty map when it is missing or
// does not parse (a corrupt cache is ignored).
std::map<std::string, TuneEntry> read_cache_file(const std::string &path)
{
    std::map<std::string, TuneEntry> parsed;
    if (path.empty()) return parsed;
    FILE *f = fopen(path.c_str(), "rb");
    if (!f) return parsed;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
    fclose(f);
    if (!parse_cache(text, parsed)) parsed.clear();
    return parsed;
}

void load_cache_locked()
{
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    g_cache = read_cache_file(cache_path());
}

void mkdirs(const std::string &dir)
{
    for (size_t pos = 1; pos <= dir.size(); ++pos)
        if (pos == dir.size() || dir[pos] == '/') mkdir(dir.substr(0, pos).c_str(), 0755);
}

// Best effort: merge with what is on disk now (other processes may have
// added entries since this one read the file; this process's entries win)
// and replace the file atomically.
void store_cache_locked(const std::string &key, const TuneEntry &e)
{
    g_cache[key] = e;
    const std::string path = cache_path();
    if (path.empty()) return;
    for (const auto &kv : read_cache_file(path)) g_cache.insert(kv);  // keeps existing keys
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) mkdirs(path.substr(0, slash));
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return;
    fprintf(f, "{\n");
    size_t k = 0;
    for (const auto &kv : g_cache)
        fprintf(f, "  \"%s\": {\"bu\": %d, \"order\": %d, \"sched\": %d, \"ms\": %.4f}%s\n",
                kv.first.c_str(), kv.second.bu, kv.second.order, kv.second.sched, kv.second.ms,
                ++k < g_cache.size() ? "," : "");
    fprintf(f, "}\n");
    if (fclose(f) == 0) rename(tmp.c_str(), path.c_str());
    else remove(tmp.c_str());
}

uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull)
{
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    return h;
}

}  // namespace

struct gpp_plan {
    int device = -1;
    int nstates = 0, nw = 0;
    std::vector<gpp::Dims32> dims;  // caller order
    std::vector<long> tiles;        // per state, caller order
    long total_tiles = 0;
    std::vector<Candidate> cands;
    int chosen = -1;
    double tuned_ms = 0.0;
    bool from_cache = false;
    std::string key;
    size_t ws_bytes = 0;
    int max_waves = 0;
    bool forced = false;  // candidates restricted by GPP_BATCHED_SCHEDULE/_BANDS
    // descriptor table (nstates + 1 entries, then kXcdCount + 1 chunk
    // boundaries): device copy, pinned staging, event guarding reuse
    gpp::StateDesc *d_desc = nullptr, *h_desc = nullptr;
    long *d_chunks = nullptr, *h_chunks = nullptr;
    size_t desc_bytes = 0;
    hipEvent_t staged = nullptr;
    int desc_cand = -1;
    std::vector<gpp_inputs> uploaded;
    // captured graph and the arguments it was captured with
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *g_ach = nullptr, *g_asx = nullptr, *g_ws = nullptr;
    int g_cand = -1;
};

namespace {

using gpp::fail;
using gpp::hip_fail;

std::vector<int> schedule(const gpp_plan *pl, int order)
{
    std::vector<int> perm(pl->nstates);
    for (int i = 0; i < pl->nstates; ++i) perm[i] = i;
    if (order == 1)
        std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
            return pl->dims[a].nb + pl->dims[a].nv > pl->dims[b].nb + pl->dims[b].nv;
        });
    return perm;
}

bool same_inputs(const gpp_inputs &a, const gpp_inputs &b)
{
    return a.aqsmtemp == b.aqsmtemp && a.aqsntemp == b.aqsntemp &&
           a.I_eps_array == b.I_eps_array && a.wtilde_array == b.wtilde_array &&
           a.vcoul == b.vcoul && a.wx_array == b.wx_array;
}

// Chunk boundaries for the XCD-chunked schedule: the tile list (schedule
// order) split at equal shares of its cost, one share per XCD in
// proportion to the waves that XCD holds (workgroups go to XCDs
// round-robin).
void xcd_chunks(const gpp_plan *pl, const std::vector<int> &perm, int blocks, long *out)
{
    const int X = gpp::kXcdCount;
    double total = 0.0;
    for (int s : perm) total += pl->tiles[s] * (pl->dims[s].nb + pl->dims[s].nv + kTileOverheadBands);
    out[0] = 0;
    double acc_share = 0.0, before = 0.0;
    long tb = 0;
    size_t k = 0;
    for (int x = 1; x < X; ++x) {
        const int per = blocks / X, rem = blocks % X;
        acc_share += (double)(per + (x - 1 < rem ? 1 : 0)) / blocks;
        const double target = acc_share * total;
        // advance whole states while their end is below the target
        while (k < perm.size()) {
            const int s = perm[k];
            const double c = pl->dims[s].nb + pl->dims[s].nv + kTileOverheadBands;
            const double end = before + pl->tiles[s] * c;
            if (end >= target) {
                long inside = (long)((target - before) / c + 0.5);
                out[x] = std::min(tb + std::max(inside, 0L), tb + pl->tiles[s]);
                break;
            }
            before = end;
            tb += pl->tiles[s];
            ++k;
        }
        if (k == perm.size()) out[x] = tb;
        if (out[x] < out[x - 1]) out[x] = out[x - 1];
    }
    out[X] = pl->total_tiles;
}

// Queue regions for the per-XCD queues: the chunk list split at equal cost
// shares (chunk costs from their states), one region per XCD.
void queue_regions(const gpp_plan *pl, const std::vector<int> &perm, long *out)
{
    const int X = gpp::kXcdCount;
    double total = 0.0;
    for (int s : perm) total += pl->tiles[s] * (pl->dims[s].nb + pl->dims[s].nv + kTileOverheadBands);
    out[0] = 0;
    long cb = 0;
    double before = 0.0;
    size_t k = 0;
    for (int x = 1; x < X; ++x) {
        const double target = total * x / X;
        out[x] = -1;
        while (k < perm.size()) {
            const int s = perm[k];
            const double c = pl->dims[s].nb + pl->dims[s].nv + kTileOverheadBands;
            const long nch = (pl->tiles[s] + kQueueChunkTiles - 1) / kQueueChunkTiles;
            const double end = before + pl->tiles[s] * c;
            if (end >= target) {
                const long inside = (long)((target - before) / (c * kQueueChunkTiles) + 0.5);
                out[x] = cb + std::min(std::max(inside, 0L), nch);
                break;
            }
            before = end;
            cb += nch;
            ++k;
        }
        if (out[x] < 0) out[x] = cb;
        if (out[x] < out[x - 1]) out[x] = out[x - 1];
    }
    long total_chunks = 0;
    for (int s : perm) total_chunks += (pl->tiles[s] + kQueueChunkTiles - 1) / kQueueChunkTiles;
    out[X] = total_chunks;
}

// Partial rows per state (schedule order) of a static schedule: the waves
// that walk a range of the tile list with stride W meet min(W, L) of a
// state's L tiles in that range first, and each of them writes one row
// (the kernel numbers them the same way, static_slot in gpp_batched.hip).
// Round-robin: one range, the whole list, W = all waves; XCD chunks: one
// range per XCD, W = that XCD's waves.  The total is at most the tile count.
std::vector<long> static_slots(const gpp_plan *pl, const std::vector<int> &perm, int blocks,
                               int sched)
{
    const int X = gpp::kXcdCount;
    std::vector<long> out(perm.size(), 0);
    long xc[gpp::kXcdCount + 1];
    if (sched == gpp::kSchedXcdChunks) xcd_chunks(pl, perm, blocks, xc);
    const long per = blocks / X, rem = blocks % X;
    long b = 0;
    for (size_t k = 0; k < perm.size(); ++k) {
        const long n = pl->tiles[perm[k]], e = b + n;
        if (sched == gpp::kSchedXcdChunks) {
            for (int x = 0; x < X; ++x) {
                const long lo = std::max(b, xc[x]), hi = std::min(e, xc[x + 1]);
                const long wx = (per + (x < rem ? 1 : 0)) * 4;
                if (hi > lo) out[k] += std::min(wx, hi - lo);
            }
        } else {
            out[k] = std::min((long)blocks * 4, n);
        }
        b = e;
    }
    return out;
}

gpp_status upload(gpp_plan *pl, int cand, const gpp_inputs *in, hipStream_t st)
{
    const int order = pl->cands[cand].order;
    if (pl->desc_cand == cand && (int)pl->uploaded.size() == pl->nstates) {
        bool same = true;
        for (int s = 0; s < pl->nstates && same; ++s) same = same_inputs(pl->uploaded[s], in[s]);
        if (same) return GPP_OK;
    }
    hipError_t e = hipEventSynchronize(pl->staged);  // the previous copy has read the staging
    if (e != hipSuccess) return hip_fail(e, "gpp_sigma_batched: staging event");
    const std::vector<int> perm = schedule(pl, order);
    const int sched = pl->cands[cand].sched;
    const bool is_static = sched == gpp::kSchedRoundRobin || sched == gpp::kSchedXcdChunks;
    const std::vector<long> slots =
        is_static ? static_slots(pl, perm, pl->cands[cand].blocks, sched) : std::vector<long>();
    long tb = 0, cb = 0;
    for (int k = 0; k < pl->nstates; ++k) {
        const int s = perm[k];
        const gpp::Dims32 &d = pl->dims[s];
        gpp::StateDesc &o = pl->h_desc[k];
        o.aqsm = reinterpret_cast<const double2 *>(in[s].aqsmtemp);
        o.aqsn = reinterpret_cast<const double2 *>(in[s].aqsntemp);
        o.ieps = reinterpret_cast<const double2 *>(in[s].I_eps_array);
        o.wt = reinterpret_cast<const double2 *>(in[s].wtilde_array);
        o.vcoul = in[s].vcoul;
        o.wx = in[s].wx_array;
        o.nb = d.nb;
        o.nv = d.nv;
        o.ng = d.ng;
        o.np = d.np;
        o.tile_begin = tb;
        o.chunk_begin = cb;
        o.out_index = s;
        o.pad = 0;
        tb += pl->tiles[s];
        // partial rows: the state's workgroups (flat form), work-queue
        // chunks, or static-schedule slots
        cb += sched == gpp::kSchedFlat ? flat_workgroups(d)
              : is_static             ? slots[k]
                                      : (pl->tiles[s] + kQueueChunkTiles - 1) / kQueueChunkTiles;
    }
    memset(&pl->h_desc[pl->nstates], 0, sizeof(gpp::StateDesc));
    pl->h_desc[pl->nstates].tile_begin = tb;
    pl->h_desc[pl->nstates].chunk_begin = cb;
    xcd_chunks(pl, perm, pl->cands[cand].blocks, pl->h_chunks);
    queue_regions(pl, perm, pl->h_chunks + gpp::kXcdCount + 1);
    if ((e = hipMemcpyAsync(pl->d_desc, pl->h_desc, pl->desc_bytes, hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipEventRecord(pl->staged, st)) != hipSuccess)
        return hip_fail(e, "gpp_sigma_batched: descriptor upload");
    pl->desc_cand = cand;
    pl->uploaded.assign(in, in + pl->nstates);
    return GPP_OK;
}

hipError_t run(gpp_plan *pl, int c, double *ach, double *asx, void *ws, hipStream_t st)
{
    const Candidate &k = pl->cands[c];
    gpp::BatchedLaunch L;
    L.nw = pl->nw;
    L.bu = k.bu;
    L.blocks = k.blocks;
    L.sched = k.sched;
    L.desc = pl->d_desc;
    L.nstates = pl->nstates;
    L.total_tiles = pl->total_tiles;
    L.xcd_chunks = pl->d_chunks;
    L.queue_begin = pl->d_chunks + gpp::kXcdCount + 1;
    L.nchunks = k.nchunks;
    L.chunk_tiles = kQueueChunkTiles;
    L.counter = static_cast<unsigned long long *>(ws);
    L.partials = reinterpret_cast<double *>(static_cast<char *>(ws) + kPartialsOffset);
    return gpp::launch_batched(L, reinterpret_cast<double2 *>(ach),
                               reinterpret_cast<double2 *>(asx), st);
}

gpp_status tune(gpp_plan *pl, const gpp_inputs *in, double *ach, double *asx, void *ws,
                hipStream_t st)
{
    if (!pl->forced) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        load_cache_locked();
        auto it = g_cache.find(pl->key);
        if (it != g_cache.end())
            for (size_t c = 0; c < pl->cands.size(); ++c)
                if (pl->cands[c].bu == it->second.bu && pl->cands[c].order == it->second.order &&
                    pl->cands[c].sched == it->second.sched) {
                    pl->chosen = (int)c;
                    pl->tuned_ms = it->second.ms;
                    pl->from_cache = true;
                    return GPP_OK;
                }
    }
    const char *mode = getenv("GPP_AUTOTUNE");
    if (mode && strcmp(mode, "off") == 0) {
        pl->chosen = 0;  // the first candidate is the default
        return GPP_OK;
    }
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return hip_fail(e, "gpp_sigma_batched: tuning events");
    }
    int best = -1;
    float best_ms = 0.0f;
    gpp_status s = GPP_OK;
    for (size_t c = 0; c < pl->cands.size() && s == GPP_OK; ++c) {
        if ((s = upload(pl, (int)c, in, st)) != GPP_OK) break;
        float ms = 0.0f;
        if ((e = run(pl, (int)c, ach, asx, ws, st)) != hipSuccess ||  // warm-up
            (e = hipEventRecord(a, st)) != hipSuccess ||
            (e = run(pl, (int)c, ach, asx, ws, st)) != hipSuccess ||
            (e = hipEventRecord(b, st)) != hipSuccess || (e = hipEventSynchronize(b)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) {
            s = hip_fail(e, "gpp_sigma_batched: tuning run");
            break;
        }
        if (getenv("GPP_TUNE_VERBOSE"))
            fprintf(stderr, "[gpp tune] %s cand %zu: bands=%d order=%d schedule=%d waves=%d %.3f ms\n",
                    pl->key.c_str(), c, pl->cands[c].bu, pl->cands[c].order, pl->cands[c].sched,
                    pl->cands[c].blocks * 4, ms);
        if (best < 0 || ms < best_ms) {
            best = (int)c;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (s != GPP_OK) return s;
    pl->chosen = best;
    pl->tuned_ms = best_ms;
    TuneEntry t;
    t.bu = pl->cands[best].bu;
    t.order = pl->cands[best].order;
    t.sched = pl->cands[best].sched;
    t.ms = best_ms;
    if (pl->forced) return GPP_OK;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    store_cache_locked(pl->key, t);
    return GPP_OK;
}

gpp_status ensure_graph(gpp_plan *pl, double *ach, double *asx, void *ws)
{
    if (pl->exec && pl->g_ach == ach && pl->g_asx == asx && pl->g_ws == ws &&
        pl->g_cand == pl->chosen)
        return GPP_OK;
    if (pl->exec) {
        (void)hipGraphExecDestroy(pl->exec);
        pl->exec = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "gpp_sigma_batched: begin capture");
    const hipError_t le = run(pl, pl->chosen, ach, asx, ws, pl->cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(pl->cap_stream, &graph);  // always end the capture
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le, "gpp_sigma_batched: captured launch");
    }
    if (e != hipSuccess) return hip_fail(e, "gpp_sigma_batched: end capture");
    e = hipGraphInstantiate(&pl->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        pl->exec = nullptr;
        return hip_fail(e, "gpp_sigma_batched: instantiate");
    }
    pl->g_ach = ach;
    pl->g_asx = asx;
    pl->g_ws = ws;
    pl->g_cand = pl->chosen;
    return GPP_OK;
}

void release(gpp_plan *pl)
{
    if (!pl) return;
    if (pl->staged) (void)hipEventSynchronize(pl->staged);
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    if (pl->staged) (void)hipEventDestroy(pl->staged);
    if (pl->d_desc) (void)hipFree(pl->d_desc);
    if (pl->h_desc) (void)hipHostFree(pl->h_desc);
    delete pl;
}

}  // namespace

extern "C" {

gpp_status gpp_plan_create(int32_t nstates, const gpp_dims *dims_host, gpp_plan **out)
{
    gpp::g_last_error[0] = '\0';
    if (!out) return fail(GPP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (nstates < 1 || nstates > GPP_MAX_STATES)
        return fail(GPP_ERR_INVALID, "nstates=%d outside [1, %d]", nstates, GPP_MAX_STATES);
    if (!dims_host) return fail(GPP_ERR_INVALID, "dims is NULL");
    gpp_plan *pl = new (std::nothrow) gpp_plan;
    if (!pl) return fail(GPP_ERR_NOMEM, "plan allocation");
    pl->nstates = nstates;
    pl->dims.resize(nstates);
    pl->tiles.resize(nstates);
    for (int s = 0; s < nstates; ++s) {
        gpp_status st = gpp::check_dims(&dims_host[s], &pl->dims[s]);
        if (st != GPP_OK) {
            char msg[512];
            snprintf(msg, sizeof msg, "state %d: %s", s, gpp::g_last_error);
            delete pl;
            return fail(st, "%s", msg);
        }
        const gpp::Dims32 &d = pl->dims[s];
        if (s > 0 && d.nw != pl->dims[0].nw) {
            delete pl;
            return fail(GPP_ERR_INVALID, "state %d: nfreq differs from state 0", s);
        }
        const int cols = gpp::bat_cols(d.nw);
        pl->tiles[s] = (d.nb && d.ng && d.np) ? (long)((d.ng + 63) / 64) * ((d.np + cols - 1) / cols) : 0;
        pl->total_tiles += pl->tiles[s];
    }
    pl->nw = pl->dims[0].nw;

    hipError_t e;
    hipDeviceProp_t prop;
    if (gpp_status ds = gpp::check_device("gpp_plan_create")) {
        delete pl;
        return ds;
    }
    if ((e = hipGetDevice(&pl->device)) != hipSuccess ||
        (e = hipGetDeviceProperties(&prop, pl->device)) != hipSuccess) {
        delete pl;
        return hip_fail(e, "gpp_plan_create: device query");
    }
    // candidates: bands per group (register budget allows fewer for many
    // frequencies) x schedule order; the first is the untuned default
    std::vector<int> bus;
    if (pl->nw <= 3 && gpp::bat_cols(pl->nw) == 2) bus = {2, 1};  // 3-band groups spill
    else if (pl->nw <= 3) bus = {3, 2};
    else if (pl->nw == 4) bus = {2, 1};
    else bus = {1};
    long nchunks = 0, flat_wgs = 0;
    for (int s = 0; s < nstates; ++s) {
        nchunks += (pl->tiles[s] + kQueueChunkTiles - 1) / kQueueChunkTiles;
        flat_wgs += flat_workgroups(pl->dims[s]);
    }
    // GPP_BATCHED_SCHEDULE=<n> keeps only candidates of schedule n (tests);
    // such a plan neither reads nor writes the tuning cache
    int only = -1;
    if (const char *f = getenv("GPP_BATCHED_SCHEDULE")) {
        only = atoi(f);
        pl->forced = true;
    }
    // GPP_BATCHED_BANDS=<b> keeps only the persistent candidates with b bands
    // per group (tests; the flat grid always runs the plain forward's tile)
    if (const char *f = getenv("GPP_BATCHED_BANDS")) {
        const int only_bu = atoi(f);
        std::vector<int> keep;
        for (int bu : bus)
            if (bu == only_bu) keep.push_back(bu);
        bus = keep;
        pl->forced = true;
    }
    size_t rows = 0;
    // the flat form first (the untuned default): the plain forward's tiles
    // and registers, one workgroup per four tiles
    if (flat_wgs <= 2147483647L && (only < 0 || only == gpp::kSchedFlat)) {
        Candidate c{gpp::fwd_bands(pl->nw), 1, gpp::kSchedFlat, (int)flat_wgs, flat_wgs};
        pl->cands.push_back(c);
        rows = std::max(rows, (size_t)flat_wgs);
    }
    // (schedule, order) pairs per tile variant; the queue ignores state order
    const int combos[4][2] = {{gpp::kSchedXcdQueues, 1},
                              {gpp::kSchedQueue, 1},
                              {gpp::kSchedXcdChunks, 1},
                              {gpp::kSchedRoundRobin, 1}};
    for (int bu : bus)
        for (const auto &cmb : combos) {
            if (only >= 0 && cmb[0] != only) continue;
            int per_cu = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, gpp::batched_kernel(pl->nw, bu, cmb[0]), 256, 0);
            if (e != hipSuccess || per_cu < 1) per_cu = 1;
            Candidate c{bu, cmb[1], cmb[0], per_cu * prop.multiProcessorCount, nchunks};
            pl->cands.push_back(c);
            pl->max_waves = std::max(pl->max_waves, c.blocks * 4);
            const bool queue = cmb[0] == gpp::kSchedQueue || cmb[0] == gpp::kSchedXcdQueues;
            size_t need = (size_t)nchunks;
            if (!queue) {
                need = 0;
                for (long v : static_slots(pl, schedule(pl, cmb[1]), c.blocks, cmb[0])) need += v;
            }
            rows = std::max(rows, need);
        }
    if (pl->cands.empty()) {
        delete pl;
        return fail(GPP_ERR_INVALID, "GPP_BATCHED_SCHEDULE=%d matches no candidate", only);
    }
    pl->ws_bytes = kPartialsOffset + (rows * 4 * pl->nw * sizeof(double) + 255) / 256 * 256;

    uint64_t h = fnv1a(&pl->nw, sizeof pl->nw);
    for (const auto &d : pl->dims) h = fnv1a(&d, sizeof d, h);
    char key[160];
    snprintf(key, sizeof key, "gfx950:batched:nw=%d:cols=%d:s=%d:n=%d:cus=%d:h=%016llx", pl->nw,
             gpp::bat_cols(pl->nw), gpp::kSchedCount, nstates, prop.multiProcessorCount,
             (unsigned long long)h);
    pl->key = key;

    const size_t sbytes = sizeof(gpp::StateDesc) * (nstates + 1);
    pl->desc_bytes = sbytes + sizeof(long) * 2 * (gpp::kXcdCount + 1);
    if ((e = hipMalloc(&pl->d_desc, pl->desc_bytes)) != hipSuccess ||
        (e = hipHostMalloc(&pl->h_desc, pl->desc_bytes, hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&pl->staged, hipEventDisableTiming)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
        release(pl);
        return hip_fail(e, "gpp_plan_create: resources");
    }
    pl->d_chunks = reinterpret_cast<long *>(reinterpret_cast<char *>(pl->d_desc) + sbytes);
    pl->h_chunks = reinterpret_cast<long *>(reinterpret_cast<char *>(pl->h_desc) + sbytes);
    *out = pl;
    return GPP_OK;
}

size_t gpp_plan_workspace(const gpp_plan *plan) { return plan ? plan->ws_bytes : 0; }

gpp_status gpp_plan_get_info(const gpp_plan *plan, gpp_plan_info *info)
{
    if (!plan || !info) return fail(GPP_ERR_INVALID, "plan or info is NULL");
    info->tuned = plan->chosen >= 0;
    info->from_cache = plan->from_cache;
    const Candidate &c = plan->cands[plan->chosen >= 0 ? plan->chosen : 0];
    info->bands_per_group = c.bu;
    info->schedule_order = c.order;
    info->schedule = c.sched;
    info->workgroups = c.blocks;
    info->waves = c.blocks * 4;
    info->candidates = (int)plan->cands.size();
    info->total_tiles = plan->total_tiles;
    info->tuned_ms = plan->tuned_ms;
    return GPP_OK;
}

gpp_status gpp_sigma_batched(gpp_plan *plan, const gpp_inputs *inputs_host, double *achtemp,
                             double *asxtemp, void *workspace, size_t workspace_bytes,
                             void *stream)
{
    gpp::g_last_error[0] = '\0';
    if (!plan) return fail(GPP_ERR_INVALID, "plan is NULL");
    if (!inputs_host) return fail(GPP_ERR_INVALID, "inputs is NULL");
    gpp::DevInputs unused;
    for (int s = 0; s < plan->nstates; ++s) {
        gpp_status st = gpp::check_inputs(plan->dims[s], &inputs_host[s], &unused);
        if (st != GPP_OK) {
            char msg[512];
            snprintf(msg, sizeof msg, "state %d: %s", s, gpp::g_last_error);
            return fail(st, "%s", msg);
        }
    }
    gpp_status st;
    const int64_t nout = (int64_t)plan->nstates * plan->nw;
    if ((st = gpp::check_array("achtemp", achtemp, nout, 16)) ||
        (st = gpp::check_array("asxtemp", asxtemp, nout, 16)))
        return st;
    if (!workspace || workspace_bytes < plan->ws_bytes)
        return fail(GPP_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu%s", plan->ws_bytes,
                    workspace_bytes, workspace ? "" : " (NULL)");
    if (gpp::misaligned(workspace, 256))
        return fail(GPP_ERR_INVALID, "workspace is not 256-byte aligned");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "gpp_sigma_batched: device query");
    if (dev != plan->device)
        return fail(GPP_ERR_INVALID, "plan was created on device %d, current is %d",
                    plan->device, dev);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if ((e = hipStreamIsCapturing(hs, &cs)) != hipSuccess)
        return hip_fail(e, "gpp_sigma_batched: capture query");
    if (cs != hipStreamCaptureStatusNone)
        return fail(GPP_ERR_INVALID, "stream is capturing; the plan replays its own graph");
    if (plan->chosen < 0 && (st = tune(plan, inputs_host, achtemp, asxtemp, workspace, hs)))
        return st;
    if ((st = upload(plan, plan->chosen, inputs_host, hs))) return st;
    if ((st = ensure_graph(plan, achtemp, asxtemp, workspace))) return st;
    if ((e = hipGraphLaunch(plan->exec, hs)) != hipSuccess)
        return hip_fail(e, "gpp_sigma_batched: graph launch");
    return GPP_OK;
}

void gpp_plan_destroy(gpp_plan *plan) { release(plan); }

}  // extern "C"
