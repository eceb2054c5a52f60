// porestokes C ABI: contexts, argument checking, the solve loop (Algorithm 1
// without MPI), Darcy reduction (App. C) and batching.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "porestokes.h"
#include "stopping.h"

using namespace ps;

struct pm_ctx {
    int dev = 0;
    size_t cap = 0, used = 0;  // used: bytes in use by the running call
    size_t pooled = 0;         // bytes kept for reuse between calls
    std::multimap<size_t, void *> pool;
    std::string err;
    std::unordered_map<void *, size_t> allocs;
    double *h_sums = nullptr;  // pinned host buffer for reduced sums
    size_t h_sums_n = 0;
    std::map<std::string, std::vector<int>> tune;  // autotuned (tile_x, tile_y, zc) per shape key
    bool tune_loaded = false;
    pm_stats stats{};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // persistent sweeps: barrier counters, the timeout flag, and whether this
    // device places workgroup i on XCD i mod 8 (-1: not checked yet)
    unsigned *d_bar = nullptr;
    int *d_fail = nullptr;
    int pers_ok = -1;
};

namespace {

pm_status fail(pm_ctx *ctx, pm_status s, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return s;
}

#define PM_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(ctx, PM_ERR_DEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),     \
                        __FILE__, __LINE__);                                                           \
    } while (0)

#define PM_TRY(expr)                                                                                   \
    do {                                                                                               \
        pm_status s_ = (expr);                                                                         \
        if (s_ != PM_OK) return s_;                                                                    \
    } while (0)

void release_pool(pm_ctx *ctx)
{
    for (auto &kv : ctx->pool) (void)hipFree(kv.second);
    ctx->pool.clear();
    ctx->pooled = 0;
}

// Device memory of a call.  Blocks that earlier calls released stay with the
// context and are handed out again when a request fits one within 1/8 of its
// size: repeated solves then skip hipMalloc (page mapping) and hipFree (a
// device-wide wait).  The pool goes back to the device when the cap or the
// device runs short, on pm_trim and on pm_destroy.
pm_status dalloc(pm_ctx *ctx, size_t bytes, void **out)
{
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    auto hit = ctx->pool.lower_bound(bytes);
    if (hit != ctx->pool.end() && hit->first - bytes <= bytes / 8) {
        const size_t got = hit->first;
        *out = hit->second;
        ctx->pool.erase(hit);
        ctx->pooled -= got;
        bytes = got;
    } else {
        if (ctx->cap && ctx->used + ctx->pooled + bytes > ctx->cap) release_pool(ctx);
        if (ctx->cap && ctx->used + bytes > ctx->cap)
            return fail(ctx, PM_ERR_OOM, "device allocation of %zu bytes exceeds the context cap (%zu used of %zu)",
                        bytes, ctx->used, ctx->cap);
        hipError_t e = hipMalloc(out, bytes);
        if (e != hipSuccess && ctx->pooled) {
            (void)hipGetLastError();
            release_pool(ctx);
            e = hipMalloc(out, bytes);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *out = nullptr;
            return fail(ctx, PM_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        }
    }
    ctx->allocs[*out] = bytes;
    ctx->used += bytes;
    if ((int64_t)ctx->used > ctx->stats.peak_bytes) ctx->stats.peak_bytes = (int64_t)ctx->used;
    return PM_OK;
}

// Return a block of dalloc to the pool.  The caller has finished every
// kernel and copy that uses it.
void dfree(pm_ctx *ctx, void *p)
{
    if (!p) return;
    auto it = ctx->allocs.find(p);
    if (it == ctx->allocs.end()) return;
    ctx->used -= it->second;
    ctx->pool.emplace(it->second, p);
    ctx->pooled += it->second;
    ctx->allocs.erase(it);
}

// Device allocations owned by one call, released on every exit path.
struct Scratch {
    pm_ctx *ctx;
    std::vector<void *> ptrs;
    explicit Scratch(pm_ctx *c) : ctx(c) {}
    ~Scratch()
    {
        if (ptrs.empty()) return;
        // an error return may leave work queued that reads these blocks: let
        // it finish before another call can be handed them
        (void)hipDeviceSynchronize();
        (void)hipGetLastError();
        for (void *p : ptrs) dfree(ctx, p);
    }
    pm_status get(size_t bytes, void **out)
    {
        pm_status s = dalloc(ctx, bytes, out);
        if (s == PM_OK) ptrs.push_back(*out);
        return s;
    }
};

pm_status ensure_host_sums(pm_ctx *ctx, size_t n)
{
    if (ctx->h_sums_n >= n) return PM_OK;
    if (ctx->h_sums) (void)hipHostFree(ctx->h_sums);
    ctx->h_sums = nullptr;
    ctx->h_sums_n = 0;
    void *p = nullptr;
    PM_HIP(hipHostMalloc(&p, n * sizeof(double), hipHostMallocDefault));
    ctx->h_sums = (double *)p;
    ctx->h_sums_n = n;
    return PM_OK;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void stats_begin(pm_ctx *ctx)
{
    std::memset(&ctx->stats, 0, sizeof ctx->stats);
    ctx->stats.total_ms = -now_ms();
    ctx->stats.peak_bytes = (int64_t)ctx->used;
}

void stats_end(pm_ctx *ctx) { ctx->stats.total_ms += now_ms(); }

// Buffers of the persistent sweeps, and the check that the dispatcher places
// workgroup i on XCD i mod 8 (the XCD of each workgroup of a 64-workgroup
// launch, from the hardware's XCC id): without it the path stays off.
pm_status ensure_pers(pm_ctx *ctx, hipStream_t s)
{
    if (ctx->pers_ok >= 0) return PM_OK;
    ctx->pers_ok = 0;
    PM_HIP(hipMalloc(&ctx->d_bar, kPersXcds * kBarrierStride * sizeof(unsigned)));
    PM_HIP(hipMalloc(&ctx->d_fail, sizeof(int)));
    PM_HIP(hipMemsetAsync(ctx->d_fail, 0, sizeof(int), s));
    static_assert(kXccProbeBlocks <= kPersXcds * kBarrierStride, "probe output must fit the counters");
    PM_HIP(launch_xcc_ids(ctx->d_bar, s));
    unsigned ids[kXccProbeBlocks];
    PM_HIP(hipMemcpyAsync(ids, ctx->d_bar, sizeof ids, hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    bool ok = true;
    for (int i = 0; i < kXccProbeBlocks; ++i) ok = ok && ids[i] == ids[i % kPersXcds];
    for (int i = 0; i < kPersXcds; ++i)
        for (int j = 0; j < i; ++j) ok = ok && ids[i] != ids[j];
    ctx->pers_ok = ok ? 1 : 0;
    return PM_OK;
}

pm_status ensure_events(pm_ctx *ctx)
{
    for (int i = 0; i < 4; ++i)
        if (!ctx->ev[i]) PM_HIP(hipEventCreate(&ctx->ev[i]));
    return PM_OK;
}

// Time a run of consecutive sweep launches: call with start=true before the
// first launch and start=false after the last; accumulates into ctx->stats.
pm_status stats_mark(pm_ctx *ctx, hipStream_t s, bool start, int64_t launches = 0, int64_t voxels = 0)
{
    PM_TRY(ensure_events(ctx));
    PM_HIP(hipEventRecord(ctx->ev[start ? 0 : 1], s));
    if (!start) {
        PM_HIP(hipEventSynchronize(ctx->ev[1]));
        float ms = 0.f;
        PM_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
        ctx->stats.sweep_ms += ms;
        ctx->stats.sweep_launches += launches;
        ctx->stats.voxel_updates += voxels;
    }
    return PM_OK;
}

pm_status check_dims(pm_ctx *ctx, int64_t nx, int64_t ny, int64_t nz)
{
    if (nx < 1 || ny < 1 || nz < 1) return fail(ctx, PM_ERR_ARG, "dims must be >= 1 (got %lld %lld %lld)",
                                                 (long long)nx, (long long)ny, (long long)nz);
    // a z-plane of a field stays below 2^31 bytes (the sweeps address one plane
    // of a field with 32-bit byte offsets)
    if (nx > (1 << 30) || ny > (1 << 30) || nz > (1 << 30) || nx * ny > (int64_t(1) << 28) ||
        nx * ny * nz > (int64_t(1) << 40))
        return fail(ctx, PM_ERR_ARG, "dims too large (%lld %lld %lld)", (long long)nx, (long long)ny,
                    (long long)nz);
    return PM_OK;
}

pm_status check_params(pm_ctx *ctx, const pm_params *p)
{
    if (!p) return fail(ctx, PM_ERR_ARG, "params is NULL");
    if (!(p->re > 0) || !(p->c2 > 0) || !(p->dt > 0) || !(p->tol > 0) || !(p->drive > 0) ||
        !std::isfinite(p->re) || !std::isfinite(p->c2) || !std::isfinite(p->dt) || !std::isfinite(p->drive))
        return fail(ctx, PM_ERR_ARG, "re, c2, dt, tol and drive must be positive and finite");
    if (p->check_every < 1) return fail(ctx, PM_ERR_ARG, "check_every must be >= 1");
    if (p->max_sweeps < 0) return fail(ctx, PM_ERR_ARG, "max_sweeps must be >= 0");
    if (p->precision < PM_FP64 || p->precision > PM_FP32_DC) return fail(ctx, PM_ERR_ARG, "bad precision");
    if (p->stop_rule != 0 && p->stop_rule != 1) return fail(ctx, PM_ERR_ARG, "bad stop_rule");
    if (p->kernel < PM_KERNEL_AUTO || p->kernel > PM_KERNEL_SIMPLE) return fail(ctx, PM_ERR_ARG, "bad kernel");
    if (p->tile_x || p->tile_y) {
        const bool f64 = p->precision != PM_FP32, f32 = p->precision != PM_FP64;
        if ((f64 && !fused_tile_supported(p->tile_x, p->tile_y, kF64)) ||
            (f32 && !fused_tile_supported(p->tile_x, p->tile_y, kF32)))
            return fail(ctx, PM_ERR_ARG, "unsupported tile %dx%d for this precision", p->tile_x, p->tile_y);
    }
    if (p->zchunk < 0) return fail(ctx, PM_ERR_ARG, "zchunk must be >= 0");
    if (p->graphs != 0 && p->graphs != 1) return fail(ctx, PM_ERR_ARG, "graphs must be 0 or 1");
    if (p->progress < 0) return fail(ctx, PM_ERR_ARG, "progress must be >= 0");
    if (p->pore_cleanup != 0 && p->pore_cleanup != 1) return fail(ctx, PM_ERR_ARG, "pore_cleanup must be 0 or 1");
    if (p->outer_walls < 0 || p->outer_walls > 7) return fail(ctx, PM_ERR_ARG, "outer_walls must be a bit mask 0..7");
    if (p->dc_form != 0 && p->dc_form != 1) return fail(ctx, PM_ERR_ARG, "dc_form must be 0 or 1");
    if (p->tblock < 0 || p->tblock > 2) return fail(ctx, PM_ERR_ARG, "tblock must be 0 (auto), 1 or 2");
    if (p->tile2_x || p->tile2_y) {
        const bool f64 = p->precision != PM_FP32, f32 = p->precision != PM_FP64;
        if ((f64 && !fused2_tile_supported(p->tile2_x, p->tile2_y, kF64)) ||
            (f32 && !fused2_tile_supported(p->tile2_x, p->tile2_y, kF32)))
            return fail(ctx, PM_ERR_ARG, "unsupported two-sweep tile %dx%d", p->tile2_x, p->tile2_y);
    }
    if (p->zchunk2 < 0) return fail(ctx, PM_ERR_ARG, "zchunk2 must be >= 0");
    if (p->fixed_pressure != 0 && p->fixed_pressure != 1)
        return fail(ctx, PM_ERR_ARG, "fixed_pressure must be 0 or 1");
    if (p->persistent != 0 && p->persistent != 1) return fail(ctx, PM_ERR_ARG, "persistent must be 0 or 1");
    return PM_OK;
}

pm_status set_device(pm_ctx *ctx)
{
    PM_HIP(hipSetDevice(ctx->dev));
    return PM_OK;
}

// ------------------------------------------------------------------ tuning

std::string tune_key(int nx, int ny, int nz, Prec prec)
{
    return std::to_string(nx) + "x" + std::to_string(ny) + "x" + std::to_string(nz) + (prec == kF64 ? ":f64" : ":f32");
}

// Tuning cache file: a flat JSON object {"NXxNYxNZ:f64": [tx, ty, zc, tb, ox, oy, zc2], ...}
// (entries of three numbers, [tx, ty, zc], are single-step choices).
void load_tune_cache(pm_ctx *ctx)
{
    const char *path = std::getenv("PORESTOKES_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    size_t pos = 0;
    for (;;) {
        size_t k0 = text.find('"', pos);
        if (k0 == std::string::npos) break;
        size_t k1 = text.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        size_t b0 = text.find('[', k1);
        if (b0 == std::string::npos) break;
        size_t b1 = text.find(']', b0);
        if (b1 == std::string::npos) break;
        std::vector<int> vals;
        const char *q = text.c_str() + b0 + 1, *qe = text.c_str() + b1;
        while (q < qe) {
            char *end = nullptr;
            const long v = std::strtol(q, &end, 10);
            if (end == q) {
                ++q;
                continue;
            }
            vals.push_back((int)v);
            q = end;
        }
        if (vals.size() == 3 || vals.size() == 7) ctx->tune[text.substr(k0 + 1, k1 - k0 - 1)] = vals;
        pos = b1 + 1;
    }
}

void save_tune_cache(const pm_ctx *ctx)
{
    const char *path = std::getenv("PORESTOKES_TUNE_CACHE");
    if (!path || !*path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{");
    bool first = true;
    for (const auto &kv : ctx->tune) {
        if (kv.second.size() != 3 && kv.second.size() != 7) continue;
        std::fprintf(f, "%s\n  \"%s\": [", first ? "" : ",", kv.first.c_str());
        for (size_t i = 0; i < kv.second.size(); ++i) std::fprintf(f, "%s%d", i ? ", " : "", kv.second[i]);
        std::fprintf(f, "]");
        first = false;
    }
    std::fprintf(f, "\n}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

// ------------------------------------------------------------------ tiles

struct TileCfg {
    int tx = 64, ty = 8, zc = 32;      // single-step kernel: tile and z-chunk
    int tb = 1;                        // sweeps per pass of the bulk launches (1 or 2)
    int ox = 64, oy = 10, zc2 = 32;    // tb = 2: output tile and z-chunk of the two-step kernel
};

int auto_zc(int nx, int ny, int nz, int tx, int ty)
{
    const int64_t txy = (int64_t)((nx + tx - 1) / tx) * ((ny + ty - 1) / ty);
    // aim for 512 * 512 threads in flight (512 workgroups of 512 threads, 256 of
    // 1024: at least one 16-wave group per CU) while keeping chunks long enough
    // to amortise priming the z window (each chunk also reads the planes just
    // below and above it); chunks of up to 64 planes measured best (16 to 256
    // tried)
    int64_t zc = (int64_t)nz * txy * tx * ty / (512LL * 512LL);
    // small grids cannot fill the chip even with 16-plane chunks: there the sweep
    // is latency-bound (one plane after another per workgroup), so shorter chunks
    // and more workgroups win and the priming bytes do not matter (32^3, FP64:
    // 9.5, 7.2 and 6.0 us per sweep with chunks of 4, 2 and 1 planes)
    zc = zc < 16 ? std::max<int64_t>(1, zc) : std::min<int64_t>(64, zc);
    return (int)std::min<int64_t>(zc, nz);
}

// z-chunk of the two-step kernel: its workgroups run one per CU (256 at a time)
// and a chunk of zc planes costs about zc + 5 stage-1 plane steps (the chunk,
// four planes beyond its ends, the prologue).  Pick the chunk that minimises
// rounds x steps, the longer chunk on ties.
int auto_zc2(int nx, int ny, int nz, int ox, int oy)
{
    const int64_t txy = (int64_t)((nx + ox - 1) / ox) * ((ny + oy - 1) / oy);
    int best = std::min(nz, 4);
    int64_t best_cost = INT64_MAX;
    for (int zc = 4; zc <= std::min(nz, 64); ++zc) {
        const int64_t chunks = (nz + zc - 1) / zc;
        const int64_t rounds = (txy * chunks + 255) / 256;
        const int64_t cost = rounds * (zc + 5);
        if (cost <= best_cost) {
            best_cost = cost;
            best = zc;
        }
    }
    return std::min(best, nz);
}

// Default output tile of the two-step kernel: 64 x 8 (68 x 12 threads) in both
// precisions, the fastest of 64x10, 64x8, 64x6, 32x24, 32x12 and 32x8 on the
// 256^3 packing (FP32 262 us, FP64 450 us per two-sweep launch).
void default_tile2(Prec prec, int *ox, int *oy)
{
    (void)prec;
    *ox = 64;
    *oy = 8;
}

TileCfg pick_tiles(pm_ctx *ctx, const pm_params *prm, int nx, int ny, int nz, Prec prec)
{
    TileCfg c;
    default_tile2(prec, &c.ox, &c.oy);
    c.zc2 = 0;
    auto it = ctx->tune.find(tune_key(nx, ny, nz, prec));
    if (it != ctx->tune.end() && (it->second.size() == 3 || it->second.size() == 7)) {
        c.tx = it->second[0];
        c.ty = it->second[1];
        c.zc = it->second[2];
        if (it->second.size() == 7) {
            c.tb = it->second[3];
            c.ox = it->second[4];
            c.oy = it->second[5];
            c.zc2 = it->second[6];
        }
    } else {
        // Measured on MI355X (256^3 packing, three instances per launch):
        // 128x8 in both precisions (FP64 655 us against 654 for 64x16 and 672
        // for 64x8; FP32 374 against 384 and 403), unless 128-wide tiles pad x
        // more than 64-wide ones (nx = 150: 256 against 192 columns).  Then
        // FP64 64x8 and FP32 64x16: on small, latency-bound grids (32^3) the
        // smaller FP64 workgroups solve 25 % faster than 64x16.  Grids at most
        // 32 wide take 32x8, whose lanes all hold columns of the grid (32^3,
        // one-plane chunks: FP64 5.5 us per sweep against 6.1 with 64x8, FP32
        // 5.2 against 7.0 with 64x16).
        const int64_t pad128 = (nx + 127) / 128 * 128, pad64 = (nx + 63) / 64 * 64;
        if (nx <= 32) {
            c.tx = 32;
            c.ty = 8;
        } else if (pad128 <= pad64) {
            c.tx = 128;
            c.ty = 8;
        } else {
            c.tx = 64;
            c.ty = prec == kF64 ? 8 : 16;
        }
        c.zc = 0;
        c.tb = 1;
    }
    if (prm->tile_x && prm->tile_y) {
        c.tx = prm->tile_x;
        c.ty = prm->tile_y;
    }
    if (prm->zchunk > 0) c.zc = prm->zchunk;
    if (c.zc <= 0) c.zc = auto_zc(nx, ny, nz, c.tx, c.ty);
    c.zc = std::min(c.zc, nz);
    if (prm->tblock > 0) c.tb = prm->tblock;
    if (prm->tile2_x && prm->tile2_y) {
        c.ox = prm->tile2_x;
        c.oy = prm->tile2_y;
    }
    if (prm->zchunk2 > 0) c.zc2 = prm->zchunk2;
    if (!fused2_tile_supported(c.ox, c.oy, prec)) default_tile2(prec, &c.ox, &c.oy);
    if (c.zc2 <= 0) c.zc2 = auto_zc2(nx, ny, nz, c.ox, c.oy);
    c.zc2 = std::min(c.zc2, nz);
    return c;
}

// ------------------------------------------------------------------ engine

struct Inst {
    // problem
    const uint8_t *mask = nullptr;
    int nx = 0, ny = 0, nz = 0, axis = 0;
    int64_t N = 0;
    double dx = 1.0, mu = 1.0;
    void *user[4] = {nullptr, nullptr, nullptr, nullptr};
    pm_history *hist = nullptr;
    // derived
    uint16_t *codes = nullptr;  // packed stencil codes
    int64_t nflow = 0, nsolid = 0;
    bool no_through_flow = false;  // outer walls close the load axis
    // state
    bool dc = false;
    bool delta = false;      // correction form: set 0/1 hold e (FP32), user holds s0 (FP64)
    bool to_delta = false;   // enter the correction form after this round of checks
    void *dsrc = nullptr;    // d0 = T(s0) - s0, 4 N floats (allocated at the first use)
    double q0[3] = {0.0, 0.0, 0.0};  // flux sums of s0
    Prec prec = kF64;
    void *set[2][4] = {};
    void *internal = nullptr;
    int64_t sweeps = 0;
    // launches since the start of the current pipeline (its pressure-passthrough
    // step included): launch j of a pipeline reads field set j & 1 and writes the
    // other, whether it advances one sweep or two
    int64_t passes = 0;
    double rmin = INFINITY, qprev = -1.0;
    int stall = 0, plateau_hits = 0;
    double r_last = INFINITY;
    std::vector<double> rphase;  // residuals at the checks of the current phase
    bool active = false, needs_start = false;
    pm_status status = PM_OK;
    double kcol[3] = {0, 0, 0};
    TileCfg tile;
    int64_t nblocks = 0, partial_rows = 0;
    int64_t nblocks2 = 0;  // blocks of a two-step launch (tile.tb = 2)
    double *partials = nullptr;
};

int64_t blocks_of(const Inst &in)
{
    return (int64_t)((in.nx + in.tile.tx - 1) / in.tile.tx) * ((in.ny + in.tile.ty - 1) / in.tile.ty) *
           ((in.nz + in.tile.zc - 1) / in.tile.zc);
}

int64_t blocks2_of(const Inst &in)
{
    return (int64_t)((in.nx + in.tile.ox - 1) / in.tile.ox) * ((in.ny + in.tile.oy - 1) / in.tile.oy) *
           ((in.nz + in.tile.zc2 - 1) / in.tile.zc2);
}

// Whether the bulk launches of an instance advance two sweeps (the two-step
// kernel has no correction-form variant).
bool two_step(const Inst &in)
{
    return in.tile.tb == 2 && !in.delta && fused2_tile_supported(in.tile.ox, in.tile.oy, in.prec);
}

size_t elem(Prec p) { return p == kF64 ? sizeof(double) : sizeof(float); }

// Device-table entry of an instance (sweep n reads set n & 1 when par_off = 0 and parity = n & 1).
bool alone_of(const Inst &in)
{
    const int64_t tiles = (int64_t)((in.nx + in.tile.tx - 1) / in.tile.tx) * ((in.ny + in.tile.ty - 1) / in.tile.ty);
    return fused_alone(in.prec, in.tile.tx, in.tile.ty, tiles);
}

// Table entry of an instance for a single-step launch, or (two) for a
// two-step launch; launch j of the block reads set (passes + j) & 1.
InstDev make_dev(const Inst &in, const pm_params *prm, int64_t blk_begin, bool skip, bool two = false)
{
    InstDev d;
    d.nx = in.nx;
    d.ny = in.ny;
    d.nz = in.nz;
    d.axis = in.axis;
    const int tx = two ? in.tile.ox : in.tile.tx, ty = two ? in.tile.oy : in.tile.ty;
    const int zc = two ? in.tile.zc2 : in.tile.zc;
    d.tiles_x = (in.nx + tx - 1) / tx;
    d.tiles_y = (in.ny + ty - 1) / ty;
    d.tiles_z = (in.nz + zc - 1) / zc;
    d.zc = zc;
    d.blk_begin = blk_begin;
    d.nblocks = two ? in.nblocks2 : in.nblocks;
    d.codes = in.codes;
    for (int s = 0; s < 2; ++s)
        for (int f = 0; f < 3; ++f) d.vel[s][f] = in.set[s][f];
    d.pres[0] = in.set[0][3];
    d.pres[1] = in.set[1][3];
    d.partials = in.partials;
    d.nu = 1.0 / prm->re;
    d.dt = prm->dt;
    d.c2dt = prm->c2 * prm->dt;
    d.drive = in.delta ? 0.0 : prm->drive;  // the correction's drive is inside d0
    d.par_off = skip ? 0 : (int)(in.passes & 1);
    d.skip = skip ? 1 : 0;
    for (int f = 0; f < 4; ++f)
        d.src[f] = in.delta ? (const char *)in.dsrc + (size_t)f * in.N * sizeof(float) : nullptr;
    d.rdt = 1.0 / prm->dt;
    d.rc2dt = 1.0 / (prm->c2 * prm->dt);
    d.fixp = prm->fixed_pressure;
    d.pad = 0;
    return d;
}


struct Engine {
    pm_ctx *ctx;
    hipStream_t stream;
    const pm_params *prm;
    std::vector<Inst> &inst;
    Scratch scratch;
    // device tables
    InstDev *d_tab = nullptr;
    size_t d_tab_cap = 0;
    PartialRef *d_refs = nullptr;
    double *d_sums = nullptr;
    std::vector<InstDev> h_tab;
    std::vector<PartialRef> h_refs;

    // Captured sweep blocks, keyed by the launch sequence they replay.  A
    // graph bakes in grid sizes and table pointers, not the table contents,
    // so it stays valid while the same groups sweep; it is rebuilt when the
    // set of active instances changes.
    std::map<std::string, hipGraphExec_t> graphs;
    hipStream_t cap_stream = nullptr;

    Engine(pm_ctx *c, hipStream_t s, const pm_params *p, std::vector<Inst> &i)
        : ctx(c), stream(s), prm(p), inst(i), scratch(c) {}

    ~Engine()
    {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }

    // One decomposition per precision across a batch: the one chosen for its
    // largest instance (tuned or default), z-chunk clamped to each instance's
    // depth.  Launches then cover every active instance of a precision at
    // once with blocks of one shape.  On the foam series a mix of per-shape
    // choices ran at 98-109 GVox/s against 120-137 for any uniform one.
    std::map<int, TileCfg> batch_tile;

    void choose_batch_tiles()
    {
        batch_tile.clear();
        if (inst.size() < 2 || (prm->tile_x && prm->tile_y)) return;
        // without tuned choices every instance takes the default tile shape and
        // its own z-chunk, exactly as a single solve of it would (same iterate)
        bool tuned = false;
        for (const Inst &in : inst)
            for (Prec p : {kF32, kF64}) tuned = tuned || ctx->tune.count(tune_key(in.nx, in.ny, in.nz, p)) > 0;
        if (!tuned) return;
        const Inst *largest = nullptr;
        for (const Inst &in : inst)
            if (!largest || in.N > largest->N) largest = &in;
        for (Prec p : {kF32, kF64})
            batch_tile[(int)p] = pick_tiles(ctx, prm, largest->nx, largest->ny, largest->nz, p);
    }

    TileCfg tile_for(const Inst &in, Prec p) const
    {
        auto it = batch_tile.find((int)p);
        if (it == batch_tile.end()) return pick_tiles(ctx, prm, in.nx, in.ny, in.nz, p);
        TileCfg c = it->second;
        c.zc = std::min(c.zc, in.nz);
        c.zc2 = std::min(c.zc2, in.nz);
        return c;
    }

    pm_status prepare()
    {
        choose_batch_tiles();
        if (prm->persistent == 1) PM_TRY(ensure_pers(ctx, stream));
        // stencil codes and counts, once per distinct mask
        std::map<const void *, size_t> first_of;
        for (size_t i = 0; i < inst.size(); ++i) {
            Inst &in = inst[i];
            auto it = first_of.find(in.mask);
            if (it != first_of.end()) {
                const Inst &o = inst[it->second];
                if (o.nx == in.nx && o.ny == in.ny && o.nz == in.nz) {
                    in.codes = o.codes;
                    in.nsolid = o.nsolid;
                    continue;
                }
            } else {
                first_of[in.mask] = i;
            }
            void *p = nullptr;
            PM_TRY(scratch.get((size_t)in.N * sizeof(uint16_t), &p));
            in.codes = (uint16_t *)p;
            PM_HIP(launch_face_codes16(in.mask, in.nx, in.ny, in.nz, in.codes, stream));
        }
        void *dcount = nullptr;
        PM_TRY(scratch.get(4 * sizeof(unsigned long long) * inst.size(), &dcount));
        unsigned long long *cnt = (unsigned long long *)dcount;
        for (size_t i = 0; i < inst.size(); ++i)
            PM_HIP(launch_counts(inst[i].mask, inst[i].codes, inst[i].N, cnt + 4 * i, stream));
        std::vector<unsigned long long> hc(4 * inst.size());
        PM_HIP(hipMemcpyAsync(hc.data(), cnt, hc.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                              stream));
        PM_HIP(hipStreamSynchronize(stream));
        for (size_t i = 0; i < inst.size(); ++i) {
            Inst &in = inst[i];
            in.nsolid = (int64_t)hc[4 * i];
            in.nflow = (int64_t)hc[4 * i + 1 + in.axis];
            in.active = true;
            if (in.no_through_flow || in.nsolid == 0 || in.nflow == 0) {
                in.status = PM_ERR_NO_FLOW;
                in.active = false;
            }
        }
        // fields and partials
        int64_t total_blocks = 0;
        for (Inst &in : inst) {
            if (!in.active) continue;
            in.dc = prm->precision == PM_FP32_DC;
            in.prec = prm->precision == PM_FP64 ? kF64 : kF32;
            const Prec user_prec = prm->precision == PM_FP32 ? kF32 : kF64;
            const size_t ue = elem(user_prec);
            if (!in.user[0]) {
                void *p = nullptr;
                PM_TRY(scratch.get(4 * (size_t)in.N * ue, &p));
                for (int f = 0; f < 4; ++f) in.user[f] = (char *)p + f * (size_t)in.N * ue;
            }
            // one internal block of 4 N user-precision values: the second set
            // (FP64/FP32) or, for FP32_DC, both FP32 sets of the first phase
            PM_TRY(scratch.get(4 * (size_t)in.N * ue, &in.internal));
            if (in.dc) {
                for (int s = 0; s < 2; ++s)
                    for (int f = 0; f < 4; ++f)
                        in.set[s][f] = (char *)in.internal + (size_t)(4 * s + f) * in.N * sizeof(float);
            } else {
                for (int f = 0; f < 4; ++f) {
                    in.set[0][f] = in.user[f];
                    in.set[1][f] = (char *)in.internal + (size_t)f * in.N * ue;
                }
            }
            in.tile = tile_for(in, in.prec);
            in.nblocks = blocks_of(in);
            in.nblocks2 = blocks2_of(in);
            if (in.dc) {  // room for the FP64 phase's decomposition too
                Inst tmp = in;
                tmp.tile = tile_for(in, kF64);
                in.partial_rows = std::max(in.nblocks, blocks_of(tmp));
            } else {
                in.partial_rows = in.nblocks;
            }
            total_blocks += in.partial_rows;
        }
        if (total_blocks > 0) {
            void *p = nullptr;
            PM_TRY(scratch.get((size_t)total_blocks * kNumSums * sizeof(double), &p));
            double *base = (double *)p;
            for (Inst &in : inst)
                if (in.active) {
                    in.partials = base;
                    base += in.partial_rows * kNumSums;
                }
        }
        void *p = nullptr;
        PM_TRY(scratch.get(2 * inst.size() * sizeof(InstDev), &p));  // single- and two-step entries
        d_tab = (InstDev *)p;
        PM_TRY(scratch.get(inst.size() * sizeof(PartialRef), &p));
        d_refs = (PartialRef *)p;
        PM_TRY(scratch.get(inst.size() * kNumSums * sizeof(double), &p));
        d_sums = (double *)p;
        PM_TRY(ensure_host_sums(ctx, inst.size() * kNumSums));
        return PM_OK;
    }

    pm_status init_state()
    {
        for (Inst &in : inst) {
            if (!in.active) continue;
            const size_t ue = prm->precision == PM_FP32 ? sizeof(float) : sizeof(double);
            if (!prm->warm_start) {
                for (int f = 0; f < 4; ++f) PM_HIP(hipMemsetAsync(in.user[f], 0, (size_t)in.N * ue, stream));
            } else {
                PM_HIP(launch_zero_solid(prm->precision == PM_FP32 ? kF32 : kF64, in.codes, in.N, in.user[0],
                                         in.user[1], in.user[2], stream));
            }
            if (in.dc) {
                for (int f = 0; f < 4; ++f)
                    PM_HIP(launch_f64_to_f32((const double *)in.user[f], (float *)in.set[0][f], in.N, stream));
            }
            in.needs_start = true;
            in.passes = 0;
        }
        return PM_OK;
    }

    InstDev dev_of(const Inst &in, int64_t blk_begin, bool skip) const { return make_dev(in, prm, blk_begin, skip); }

    // Whether an instance's blocks of sweeps run as persistent launches, and
    // its decomposition there: 32x16 tiles (the smallest plane step that
    // covers a 32-wide grid) with z-chunks long enough that it takes at most
    // kPersMaxBlocks workgroups (one XCD).  Only where the two field sets and
    // the codes fit one XCD's L2 (4 MB; 3 MiB taken): beyond that one XCD's
    // share of HBM bandwidth would cost more than the launches it saves.
    bool pers_cfg(const Inst &in, int *zc, int64_t *nb) const
    {
        if (prm->persistent != 1 || ctx->pers_ok != 1 || in.delta) return false;
        const size_t ws = 8 * elem(in.prec) * (size_t)in.N + sizeof(uint16_t) * (size_t)in.N;
        if (ws > kPersL2Bytes) return false;
        const int64_t tpp = (int64_t)((in.nx + kPersTX - 1) / kPersTX) * ((in.ny + kPersTY - 1) / kPersTY);
        if (tpp > kPersMaxBlocks) return false;
        const int64_t chunks = std::min<int64_t>(in.nz, kPersMaxBlocks / tpp);
        *zc = (int)((in.nz + chunks - 1) / chunks);
        *nb = tpp * ((in.nz + *zc - 1) / *zc);
        return true;
    }

    // Advance the selected instances by `steps` sweeps (skip: the one
    // pressure-passthrough step that starts a pipeline) with the residual sums
    // of the last one, and bring the sums to ctx->h_sums in selection order.
    //
    // Launch plan per group of instances: with the two-step kernel, (steps - 1)
    // / 2 two-step launches, then one or two single steps; the last launch is
    // always a single step carrying the reduction, so that the state of the
    // check, v^n and p^n, is in memory (v^n is the last launch's input).
    // Otherwise `steps` single steps.
    pm_status run_block(const std::vector<int> &sel, int steps, bool skip)
    {
        // one sub-table per (precision, tile) group, contiguous in d_tab; the
        // two-step entries of the groups that use it follow all single-step ones
        h_tab.clear();
        h_refs.clear();
        struct Group {
            Prec prec;
            bool src, alone, two;
            int tx, ty, ox, oy;
            int first, count;
            int64_t blocks;
            int first2;
            int64_t blocks2;
            int n2, n1;  // two-step and single-step launches of the plan
            bool pers;   // the first steps - 1 sweeps as one persistent launch
            int firstp;
            int64_t maxbp;  // most workgroups of one instance in it
            int np;         // sweeps in it
        };
        std::vector<Group> groups;
        std::vector<int> order;
        for (int pass = 0; pass < 3; ++pass)  // FP32, FP32 correction form, FP64
            for (int i : sel) {
                const Inst &in = inst[i];
                if (pass != (in.prec == kF64 ? 2 : in.delta ? 1 : 0)) continue;
                const bool alone = alone_of(in);
                int pzc = 0;
                int64_t pnb = 0;
                const bool pers = !skip && steps >= 2 && pers_cfg(in, &pzc, &pnb);
                const bool two = !pers && !skip && steps >= 3 && two_step(in);
                if (groups.empty() || groups.back().prec != in.prec || groups.back().src != in.delta ||
                    groups.back().alone != alone || groups.back().tx != in.tile.tx || groups.back().ty != in.tile.ty ||
                    groups.back().two != two ||
                    (two && (groups.back().ox != in.tile.ox || groups.back().oy != in.tile.oy)) ||
                    groups.back().pers != pers || (pers && groups.back().count == kPersXcds))
                    groups.push_back({in.prec, in.delta, alone, two, in.tile.tx, in.tile.ty, in.tile.ox, in.tile.oy,
                                      (int)h_tab.size(), 0, 0, 0, 0, 0, 0, pers, 0, 0, 0});
                Group &g = groups.back();
                h_tab.push_back(dev_of(in, g.blocks, skip));
                g.blocks += in.nblocks;
                g.count++;
                order.push_back(i);
            }
        int64_t vox2 = 0;  // voxel passes of the two-step launches (two sweeps each)
        for (Group &g : groups) {
            if (g.two) {
                g.n2 = (steps - 1) / 2;
                g.n1 = steps - 2 * g.n2;
                g.first2 = (int)h_tab.size();
                for (int k = 0; k < g.count; ++k) {
                    const Inst &in = inst[order[g.first + k]];
                    h_tab.push_back(make_dev(in, prm, g.blocks2, false, true));
                    g.blocks2 += in.nblocks2;
                    vox2 += in.N * g.n2;
                }
            } else if (g.pers) {
                // instance k of the group on XCD k, its own decomposition
                g.np = steps - 1;
                g.n1 = 1;
                g.firstp = (int)h_tab.size();
                int64_t bb = 0;
                for (int k = 0; k < g.count; ++k) {
                    Inst ip = inst[order[g.first + k]];
                    int64_t nb = 0;
                    pers_cfg(ip, &ip.tile.zc, &nb);
                    ip.tile.tx = kPersTX;
                    ip.tile.ty = kPersTY;
                    ip.nblocks = nb;
                    h_tab.push_back(make_dev(ip, prm, bb, false));
                    bb += nb;
                    g.maxbp = std::max(g.maxbp, nb);
                }
            } else {
                g.n1 = steps;
            }
        }
        for (int i : order) h_refs.push_back({inst[i].partials, inst[i].nblocks});
        PM_HIP(hipMemcpyAsync(d_tab, h_tab.data(), h_tab.size() * sizeof(InstDev), hipMemcpyHostToDevice, stream));
        PM_HIP(hipMemcpyAsync(d_refs, h_refs.data(), h_refs.size() * sizeof(PartialRef), hipMemcpyHostToDevice,
                              stream));
        int64_t vox = 0;
        for (int i : order) vox += inst[i].N;
        int64_t launches = 0, launches2 = 0, launchesp = 0, sweepsp = 0;
        for (const Group &g : groups) {
            launches += g.n1 + g.n2 + (g.pers ? 1 : 0);
            launches2 += g.n2;
            if (g.pers) {
                launchesp += 1;
                sweepsp += (int64_t)g.np * g.count;
            }
        }
        PM_TRY(ensure_events(ctx));
        // the sequence, in two parts: (a) the two-step launches of every group;
        // (b) the single steps (reduce on the last), the final reduction, the
        // copy of the sums to pinned memory.  Launch j of a group reads set
        // (passes + j) & 1.  Timing events go on the caller's stream before (a),
        // between the parts and after (b); with graphs each part is one graph.
        auto enqueue_two = [&](hipStream_t st) -> pm_status {
            for (const Group &g : groups)
                for (int j = 0; j < g.n2; ++j)
                    PM_HIP(launch_fused2(g.prec, g.ox, g.oy, d_tab + g.first2, g.count, g.blocks2, j & 1, st));
            return PM_OK;
        };
        auto enqueue_one = [&](hipStream_t st) -> pm_status {
            for (const Group &g : groups) {
                if (g.pers)
                    PM_HIP(launch_fused_pers(g.prec, kPersTX, kPersTY, d_tab + g.firstp, g.count, g.maxbp, 0, g.np,
                                             ctx->d_bar, ctx->d_fail, st));
                for (int k = 0; k < g.n1; ++k) {
                    const int j = g.n2 + g.np + k;
                    const int red = k == g.n1 - 1 ? 1 : 0;
                    if (g.src)
                        PM_HIP(launch_fused_src(g.tx, g.ty, d_tab + g.first, g.count, g.blocks, j & 1, red, st,
                                                g.alone));
                    else
                        PM_HIP(launch_fused(g.prec, g.tx, g.ty, d_tab + g.first, g.count, g.blocks, j & 1, red, st,
                                            g.alone));
                }
            }
            PM_HIP(launch_reduce_partials(d_refs, (int)order.size(), d_sums, st));
            PM_HIP(hipMemcpyAsync(ctx->h_sums, d_sums, order.size() * kNumSums * sizeof(double),
                                  hipMemcpyDeviceToHost, st));
            return PM_OK;
        };
        if (prm->graphs && !skip && launchesp == 0) {
            std::string key;
            for (const Group &g : groups)
                key += "|" + std::to_string(g.prec) + (g.src ? "s" : "") + (g.alone ? "a" : "") + ":" +
                       std::to_string(g.tx) + "x" + std::to_string(g.ty) + ":" + std::to_string(g.first) + ":" +
                       std::to_string(g.count) + ":" + std::to_string(g.blocks) + ":" + std::to_string(g.n1) +
                       (g.two ? ":2:" + std::to_string(g.ox) + "x" + std::to_string(g.oy) + ":" +
                                    std::to_string(g.first2) + ":" + std::to_string(g.blocks2) + ":" +
                                    std::to_string(g.n2)
                              : "");
            key += "|" + std::to_string(order.size());
            hipGraphExec_t ex2 = nullptr, ex1 = nullptr;
            PM_TRY(graph_of("2" + key, enqueue_two, launches2 > 0, &ex2));
            PM_TRY(graph_of("1" + key, enqueue_one, true, &ex1));
            PM_HIP(hipEventRecord(ctx->ev[0], stream));
            if (ex2) PM_HIP(hipGraphLaunch(ex2, stream));
            PM_HIP(hipEventRecord(ctx->ev[2], stream));
            PM_HIP(hipGraphLaunch(ex1, stream));
            PM_HIP(hipEventRecord(ctx->ev[1], stream));
        } else {
            PM_HIP(hipEventRecord(ctx->ev[0], stream));
            PM_TRY(enqueue_two(stream));
            PM_HIP(hipEventRecord(ctx->ev[2], stream));
            PM_TRY(enqueue_one(stream));
            PM_HIP(hipEventRecord(ctx->ev[1], stream));
        }
        PM_HIP(hipStreamSynchronize(stream));
        {
            float ms = 0.f, ms2 = 0.f;
            PM_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
            PM_HIP(hipEventElapsedTime(&ms2, ctx->ev[0], ctx->ev[2]));
            ctx->stats.sweep_ms += ms;
            ctx->stats.sweep_launches += launches;
            ctx->stats.voxel_updates += vox * steps;
            if (launches2 > 0) {
                ctx->stats.t2_ms += ms2;
                ctx->stats.t2_launches += launches2;
                ctx->stats.t2_voxels += vox2;
            }
            ctx->stats.pers_launches += launchesp;
            ctx->stats.pers_sweeps += sweepsp;
            const Inst &last = inst[order.back()];
            ctx->stats.tile_x = last.tile.tx;
            ctx->stats.tile_y = last.tile.ty;
            ctx->stats.zchunk = last.tile.zc;
            ctx->stats.precision = last.prec == kF64 ? PM_FP64 : PM_FP32;
            ctx->stats.tblock = groups.back().two ? 2 : 1;
        }
        if (launchesp > 0) {
            int hf = 0;
            PM_HIP(hipMemcpy(&hf, ctx->d_fail, sizeof hf, hipMemcpyDeviceToHost));
            if (hf) {
                PM_HIP(hipMemset(ctx->d_fail, 0, sizeof(int)));
                return fail(ctx, PM_ERR_DEVICE, "persistent sweeps: a barrier wait ran out (the state is incomplete)");
            }
        }
        for (const Group &g : groups)
            for (int k = 0; k < g.count; ++k) inst[order[g.first + k]].passes += g.n1 + g.n2 + g.np;
        // h_sums rows follow `order`; remap to `sel` positions
        sums_of.assign(inst.size(), nullptr);
        for (size_t r = 0; r < order.size(); ++r) sums_of[order[r]] = ctx->h_sums + r * kNumSums;
        return PM_OK;
    }

    // The executable graph captured from `enqueue` under `key` (captured on
    // first use); none when `want` is false.
    template <typename F>
    pm_status graph_of(const std::string &key, F &&enqueue, bool want, hipGraphExec_t *out)
    {
        *out = nullptr;
        if (!want) return PM_OK;
        auto it = graphs.find(key);
        if (it == graphs.end()) {
            if (!cap_stream) PM_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
            PM_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
            pm_status es = enqueue(cap_stream);
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(cap_stream, &g);
            if (es != PM_OK) {
                if (g) (void)hipGraphDestroy(g);
                return es;
            }
            PM_HIP(ee);
            hipGraphExec_t ex = nullptr;
            hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            PM_HIP(ei);
            it = graphs.emplace(key, ex).first;
        }
        *out = it->second;
        return PM_OK;
    }
    std::vector<const double *> sums_of;

    void record(Inst &in, const double *s, double r, double eps)
    {
        for (int k = 0; k < 3; ++k)
            in.kcol[k] = s[2 + k] / ((double)in.N * prm->re * prm->drive) * in.dx * in.dx;
        pm_history *h = in.hist;
        if (h && h->n < h->cap) {
            const int64_t j = h->n++;
            if (h->sweep) h->sweep[j] = in.sweeps;
            if (h->resid) h->resid[j] = r;
            if (h->eps_q) h->eps_q[j] = eps;
            if (h->q)
                for (int k = 0; k < 3; ++k) h->q[3 * j + k] = s[2 + k] / (double)in.N;
        }
    }

    // Copy the state of the last check into the user fields.
    pm_status finalize(Inst &in)
    {
        const int vs = (int)((in.passes - 1) & 1), ps_ = (int)(in.passes & 1);
        const size_t e = elem(in.prec);
        // in the final phase set 0 is the user set (FP64, FP32) -- for FP32_DC the
        // FP32 phase never finalises with status OK, but may with an error status
        if (in.delta) {
            PM_TRY(fold_correction(in));
        } else if (in.dc && in.prec == kF32) {
            for (int f = 0; f < 3; ++f)
                PM_HIP(launch_f32_to_f64((const float *)in.set[vs][f], (double *)in.user[f], in.N, stream));
            PM_HIP(launch_f32_to_f64((const float *)in.set[ps_][3], (double *)in.user[3], in.N, stream));
        } else {
            if (vs != 0)
                for (int f = 0; f < 3; ++f)
                    PM_HIP(hipMemcpyAsync(in.user[f], in.set[vs][f], (size_t)in.N * e, hipMemcpyDeviceToDevice,
                                          stream));
            if (ps_ != 0)
                PM_HIP(hipMemcpyAsync(in.user[3], in.set[ps_][3], (size_t)in.N * e, hipMemcpyDeviceToDevice,
                                      stream));
        }
        in.active = false;
        return PM_OK;
    }

    // s0 + e into the user fields (FP64) at the end of the correction form
    pm_status fold_correction(Inst &in)
    {
        const int vs = (int)((in.passes - 1) & 1), ps_ = (int)(in.passes & 1);
        for (int f = 0; f < 3; ++f)
            PM_HIP(launch_add_f32_to_f64((const float *)in.set[vs][f], (double *)in.user[f], in.N, stream));
        PM_HIP(launch_add_f32_to_f64((const float *)in.set[ps_][3], (double *)in.user[3], in.N, stream));
        in.delta = false;
        return PM_OK;
    }

    // Start a new phase (FP64 after promotion, or the correction form): a new
    // pipeline from its own first check.  eps_q of that check must not compare
    // with the previous phase's last check, which holds the same state.
    void restart_phase(Inst &in)
    {
        in.nblocks = blocks_of(in);
        in.nblocks2 = blocks2_of(in);
        in.passes = 0;
        in.needs_start = true;
        in.rmin = INFINITY;
        in.stall = 0;
        in.plateau_hits = 0;
        in.rphase.clear();
        in.qprev = -1.0;
    }

    // FP32 phase (or correction form) -> FP64 phase from the promoted state.
    pm_status promote(Inst &in)
    {
        if (in.delta) {
            PM_TRY(fold_correction(in));
        } else {
            const int vs = (int)((in.passes - 1) & 1), ps_ = (int)(in.passes & 1);
            for (int f = 0; f < 3; ++f)
                PM_HIP(launch_f32_to_f64((const float *)in.set[vs][f], (double *)in.user[f], in.N, stream));
            PM_HIP(launch_f32_to_f64((const float *)in.set[ps_][3], (double *)in.user[3], in.N, stream));
        }
        in.prec = kF64;
        for (int f = 0; f < 4; ++f) {
            in.set[0][f] = in.user[f];
            in.set[1][f] = (char *)in.internal + (size_t)f * in.N * sizeof(double);
        }
        in.tile = tile_for(in, kF64);
        const int64_t nb = blocks_of(in);
        if (nb > in.partial_rows) return fail(ctx, PM_ERR_ARG, "internal: block count grew on promotion");
        in.nblocks = nb;
        restart_phase(in);
        return PM_OK;
    }

    // FP32 phase at its floor -> correction form (pm_params.dc_form = 0):
    // s0 to FP64 in the user fields, one FP64 sweep T(s0) into the internal
    // block (its sums give the flux of s0), d0 = T(s0) - s0 in FP32, and the
    // FP32 correction e from 0 in the internal block.  Without memory for d0
    // the state is promoted instead.
    pm_status enter_delta(int i)
    {
        Inst &in = inst[i];
        if (!in.dsrc) {
            void *p = nullptr;
            if (scratch.get(4 * (size_t)in.N * sizeof(float), &p) != PM_OK) {
                ctx->err.clear();
                ctx->stats.dc_promoted_for_memory++;
                return promote(in);
            }
            in.dsrc = p;
        }
        const int vs = (int)((in.passes - 1) & 1), ps_ = (int)(in.passes & 1);
        for (int f = 0; f < 3; ++f)
            PM_HIP(launch_f32_to_f64((const float *)in.set[vs][f], (double *)in.user[f], in.N, stream));
        PM_HIP(launch_f32_to_f64((const float *)in.set[ps_][3], (double *)in.user[3], in.N, stream));
        in.prec = kF64;
        for (int f = 0; f < 4; ++f) {
            in.set[0][f] = in.user[f];
            in.set[1][f] = (char *)in.internal + (size_t)f * in.N * sizeof(double);
        }
        in.tile = tile_for(in, kF64);
        in.nblocks = blocks_of(in);
        if (in.nblocks > in.partial_rows) return fail(ctx, PM_ERR_ARG, "internal: block count grew on promotion");
        in.passes = 0;  // the full update, reading set 0 (passes is reset with the phase below)
        PM_TRY(run_block({i}, 1, false));
        for (int k = 0; k < 3; ++k) in.q0[k] = sums_of[i][2 + k];
        for (int f = 0; f < 4; ++f)
            PM_HIP(launch_defect((const double *)in.set[1][f], (const double *)in.user[f],
                                 (float *)in.dsrc + (size_t)f * in.N, in.N, stream));
        in.prec = kF32;
        in.delta = true;
        for (int s = 0; s < 2; ++s)
            for (int f = 0; f < 4; ++f)
                in.set[s][f] = (char *)in.internal + (size_t)(4 * s + f) * in.N * sizeof(float);
        PM_HIP(hipMemsetAsync(in.internal, 0, 4 * (size_t)in.N * sizeof(float), stream));
        in.tile = tile_for(in, kF32);
        restart_phase(in);
        return PM_OK;
    }

    pm_status enter_pending()
    {
        for (int i = 0; i < (int)inst.size(); ++i)
            if (inst[i].to_delta) {
                inst[i].to_delta = false;
                if (inst[i].active) PM_TRY(enter_delta(i));
            }
        return PM_OK;
    }

    // FP32 rounding floor reached?  Two consecutive hits of the plateau
    // reading (csrc/stopping.h) on the phase's residual history.
    bool at_fp32_floor(Inst &in) const
    {
        const bool hit = plateau_reading(in.rphase.data(), in.rphase.size());
        in.plateau_hits = hit ? in.plateau_hits + 1 : 0;
        return in.plateau_hits >= 2;
    }

    // Convergence bookkeeping after a check of instance `in` with sums s.
    pm_status check(Inst &in, const double *sums)
    {
        // in the correction form the flux sums are those of e: add those of s0
        double s[kNumSums];
        for (int k = 0; k < kNumSums; ++k) s[k] = sums[k];
        const double qe = std::sqrt(s[2] * s[2] + s[3] * s[3] + s[4] * s[4]) / (double)in.N;
        if (in.delta)
            for (int k = 0; k < 3; ++k) s[2 + k] += in.q0[k];
        const double r = std::sqrt(s[0] + s[1]) / (prm->drive * std::sqrt((double)in.nflow));
        const double qn = std::sqrt(s[2] * s[2] + s[3] * s[3] + s[4] * s[4]) / (double)in.N;
        const double eps = (in.qprev >= 0.0 && qn > 0.0) ? std::fabs(qn - in.qprev) / qn : INFINITY;
        in.qprev = qn;
        record(in, s, r, eps);
        in.r_last = r;
        in.rphase.push_back(r);
        if (!std::isfinite(r) || r > 1e3 * in.rmin) {
            in.status = PM_DIVERGED;
            return finalize(in);
        }
        if (r < in.rmin) {
            in.rmin = r;
            in.stall = 0;
        } else {
            in.stall++;
        }
        const bool fp32_phase = in.prec == kF32;
        // FP32 rounding stops the velocity updates once dt |F| falls below half an
        // ulp of the velocity: r bottoms out near 2^-24 |v| / (dt G).  A plateau
        // counts only within three decades of that level (|v| from the mean flux,
        // local velocities being larger), or after 20 checks without a new minimum:
        // a slowly decelerating residual far above the floor is not the floor.
        // (in the correction form: 2^-24 |e| / (dt G))
        const double r_floor = std::ldexp(in.delta ? qe : qn, -24) / (prm->dt * prm->drive);
        const bool near_floor = r < 1e3 * r_floor;
        // the plateau test keeps a count across checks: run it only where the
        // floor decision reads it
        const bool plateau = fp32_phase && near_floor && in.stall < 5 && at_fp32_floor(in);
        CheckState c;
        c.dc = in.dc;
        c.fp32_phase = fp32_phase;
        c.delta = in.delta;
        c.stop_rule = prm->stop_rule;
        c.dc_form = prm->dc_form;
        c.tol = prm->tol;
        c.r = r;
        c.eps = eps;
        c.near_floor = near_floor;
        c.stall = in.stall;
        c.plateau = plateau;
        c.budget_spent = in.sweeps >= prm->max_sweeps;
        switch (decide(c)) {
        case CheckAction::Stop:
            in.status = PM_OK;
            return finalize(in);
        case CheckAction::NotConverged:
            in.status = PM_NOT_CONVERGED;
            return finalize(in);
        case CheckAction::Promote:
            return promote(in);
        case CheckAction::ToCorrection:
            in.to_delta = true;  // after this round of checks: it launches a sweep
            return PM_OK;
        case CheckAction::Continue:
            break;
        }
        return PM_OK;
    }

    int64_t nchecks = 0;

    pm_status run()
    {
        PM_TRY(prepare());
        PM_TRY(init_state());
        for (;;) {
            std::vector<int> starters, actives;
            for (int i = 0; i < (int)inst.size(); ++i)
                if (inst[i].active && inst[i].needs_start) starters.push_back(i);
            if (!starters.empty()) {
                PM_TRY(run_block(starters, 1, true));
                for (int i : starters) {
                    inst[i].needs_start = false;
                    PM_TRY(check(inst[i], sums_of[i]));
                }
                PM_TRY(enter_pending());
                continue;  // promotions inside the check restart their pipeline
            }
            int64_t remaining = INT64_MAX;
            for (int i = 0; i < (int)inst.size(); ++i)
                if (inst[i].active) {
                    actives.push_back(i);
                    remaining = std::min(remaining, prm->max_sweeps - inst[i].sweeps);
                }
            if (actives.empty()) break;
            // a check at every multiple of check_every and at max_sweeps
            int64_t to_next = prm->check_every - (inst[actives[0]].sweeps % prm->check_every);
            const int steps = (int)std::max<int64_t>(1, std::min(to_next, remaining));
            PM_TRY(run_block(actives, steps, false));
            double rworst = 0.0;
            for (int i : actives) {
                inst[i].sweeps += steps;
                PM_TRY(check(inst[i], sums_of[i]));
                rworst = std::max(rworst, inst[i].r_last);
            }
            PM_TRY(enter_pending());
            if (prm->progress > 0 && (++nchecks % prm->progress) == 0) {
                int nact = 0;
                for (const Inst &in : inst) nact += in.active;
                std::fprintf(stderr, "[porestokes] sweep %lld: %zu swept, %d still active, largest r %.3e\n",
                             (long long)inst[actives[0]].sweeps, actives.size(), nact, rworst);
                std::fflush(stderr);
            }
        }
        PM_HIP(hipStreamSynchronize(stream));
        return PM_OK;
    }
};

// Time every supported decomposition of the fused sweep on one shape and
// precision (from rest, on scratch fields) and keep the fastest: the
// single-step tiles and z-chunks, then the two-step tiles and z-chunks, each
// priced per sweep.  The single-step choice is kept either way (the first
// step of a pipeline and the checked steps are single steps).
pm_status autotune_shape(pm_ctx *ctx, hipStream_t s, const uint8_t *mask, int nx, int ny, int nz, Prec prec,
                         TileCfg *best_out)
{
    const int64_t N = (int64_t)nx * ny * nz;
    Scratch scratch(ctx);
    void *codes = nullptr, *fields = nullptr, *tab = nullptr, *part = nullptr;
    PM_TRY(scratch.get((size_t)N * sizeof(uint16_t), &codes));
    PM_TRY(scratch.get(8 * (size_t)N * elem(prec), &fields));
    PM_TRY(scratch.get(3 * sizeof(InstDev), &tab));
    PM_HIP(launch_face_codes16(mask, nx, ny, nz, (uint16_t *)codes, s));
    PM_HIP(hipMemsetAsync(fields, 0, 4 * (size_t)N * elem(prec), s));
    const int tiles[5][2] = {{128, 8}, {64, 8}, {32, 8}, {32, 16}, {64, 16}};
    const int tiles2[6][2] = {{64, 10}, {64, 8}, {64, 6}, {32, 24}, {32, 12}, {32, 8}};
    const int zcs[4] = {16, 32, 64, 128};
    struct Cand {
        TileCfg c;
        bool two;
    };
    std::vector<Cand> cands;
    for (auto &t : tiles) {
        if (!fused_tile_supported(t[0], t[1], prec)) continue;
        int last = -1;
        for (int zc : zcs) {
            const int z = std::min(zc, nz);
            if (z == last) continue;
            last = z;
            TileCfg c;
            c.tx = t[0];
            c.ty = t[1];
            c.zc = z;
            cands.push_back({c, false});
        }
    }
    for (auto &t : tiles2) {
        if (!fused2_tile_supported(t[0], t[1], prec)) continue;
        std::vector<int> zc2s = {auto_zc2(nx, ny, nz, t[0], t[1]), 16, 32, 64};
        std::sort(zc2s.begin(), zc2s.end());
        int last = -1;
        for (int zc : zc2s) {
            const int z = std::min(zc, nz);
            if (z == last) continue;
            last = z;
            TileCfg c;
            c.tb = 2;
            c.ox = t[0];
            c.oy = t[1];
            c.zc2 = z;
            cands.push_back({c, true});
        }
    }
    int64_t maxb = 0;
    for (const Cand &k : cands) {
        Inst in;
        in.nx = nx;
        in.ny = ny;
        in.nz = nz;
        in.tile = k.c;
        maxb = std::max(maxb, k.two ? blocks2_of(in) : blocks_of(in));
    }
    PM_TRY(scratch.get((size_t)maxb * kNumSums * sizeof(double), &part));
    pm_params prm;
    pm_params_default(&prm);
    // timed launches per candidate: ~2e9 voxel passes, at least 3
    const int reps = (int)std::max<int64_t>(3, std::min<int64_t>(20, (int64_t)2000000000 / std::max<int64_t>(N, 1)));
    PM_TRY(ensure_events(ctx));
    float best1_ms = INFINITY, best2_ms = INFINITY;  // per sweep
    TileCfg best1 = cands.front().c, best2;
    bool have2 = false;
    for (const Cand &k : cands) {
        Inst in;
        in.nx = nx;
        in.ny = ny;
        in.nz = nz;
        in.N = N;
        in.codes = (uint16_t *)codes;
        in.prec = prec;
        for (int f = 0; f < 4; ++f) {
            in.set[0][f] = (char *)fields + (size_t)f * N * elem(prec);
            in.set[1][f] = (char *)fields + (size_t)(4 + f) * N * elem(prec);
        }
        in.tile = k.two ? best1 : k.c;  // the two-step candidates start from the best single-step tile
        if (k.two) {
            in.tile.tb = 2;
            in.tile.ox = k.c.ox;
            in.tile.oy = k.c.oy;
            in.tile.zc2 = k.c.zc2;
        }
        in.nblocks = blocks_of(in);
        in.nblocks2 = blocks2_of(in);
        in.partials = (double *)part;
        InstDev d[3] = {make_dev(in, &prm, 0, true), make_dev(in, &prm, 0, false),
                        make_dev(in, &prm, 0, false, true)};
        PM_HIP(launch_store_insts(d, 3, (InstDev *)tab, s));
        InstDev *dt = (InstDev *)tab;
        const bool alone = alone_of(in);
        PM_HIP(launch_fused(prec, in.tile.tx, in.tile.ty, dt, 1, in.nblocks, 0, 0, s, alone));
        if (k.two)
            PM_HIP(launch_fused2(prec, in.tile.ox, in.tile.oy, dt + 2, 1, in.nblocks2, 1, s));
        else
            PM_HIP(launch_fused(prec, in.tile.tx, in.tile.ty, dt + 1, 1, in.nblocks, 1, 0, s, alone));
        PM_HIP(hipEventRecord(ctx->ev[0], s));
        for (int r = 0; r < reps; ++r) {
            if (k.two)
                PM_HIP(launch_fused2(prec, in.tile.ox, in.tile.oy, dt + 2, 1, in.nblocks2, r & 1, s));
            else
                PM_HIP(launch_fused(prec, in.tile.tx, in.tile.ty, dt + 1, 1, in.nblocks, r & 1, 0, s, alone));
        }
        PM_HIP(hipEventRecord(ctx->ev[1], s));
        PM_HIP(hipEventSynchronize(ctx->ev[1]));
        float ms = 0.f;
        PM_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
        const float per_sweep = ms / (k.two ? 2.0f : 1.0f);
        if (!k.two && per_sweep < best1_ms) {
            best1_ms = per_sweep;
            best1 = k.c;
        }
        if (k.two && per_sweep < best2_ms) {
            best2_ms = per_sweep;
            best2 = in.tile;
            have2 = true;
        }
    }
    TileCfg best = best1;
    best.tb = 1;
    default_tile2(prec, &best.ox, &best.oy);
    best.zc2 = auto_zc2(nx, ny, nz, best.ox, best.oy);
    if (have2) {
        best.ox = best2.ox;
        best.oy = best2.oy;
        best.zc2 = best2.zc2;
        if (best2_ms < best1_ms) best.tb = 2;
    }
    ctx->tune[tune_key(nx, ny, nz, prec)] = {best.tx, best.ty, best.zc, best.tb, best.ox, best.oy, best.zc2};
    save_tune_cache(ctx);
    if (best_out) *best_out = best;
    return PM_OK;
}

int severity(pm_status s)
{
    switch (s) {
    case PM_OK: return 0;
    case PM_NOT_CONVERGED: return 1;
    case PM_ERR_NO_FLOW: return 2;
    case PM_DIVERGED: return 3;
    default: return 4;
    }
}

pm_status check_instance_args(pm_ctx *ctx, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz, int axis,
                              double dx, double mu, void *const f[4], bool fields_required, size_t align)
{
    if (!mask) return fail(ctx, PM_ERR_ARG, "mask is NULL");
    PM_TRY(check_dims(ctx, nx, ny, nz));
    if (axis < 0 || axis > 2) return fail(ctx, PM_ERR_ARG, "axis must be 0, 1 or 2 (got %d)", axis);
    if (!(dx > 0) || !std::isfinite(dx)) return fail(ctx, PM_ERR_ARG, "voxel_size must be positive");
    if (!(mu > 0) || !std::isfinite(mu)) return fail(ctx, PM_ERR_ARG, "mu must be positive");
    int nnull = 0;
    for (int i = 0; i < 4; ++i) {
        if (!f[i]) ++nnull;
        else if (!aligned(f[i], align)) return fail(ctx, PM_ERR_ARG, "field %d is misaligned", i);
    }
    if (fields_required && nnull) return fail(ctx, PM_ERR_ARG, "field pointers must not be NULL");
    if (nnull != 0 && nnull != 4) return fail(ctx, PM_ERR_ARG, "give all four field pointers or none");
    return PM_OK;
}

// ------------------------------------------------------------ pore connectivity
//
// Which pore components wind around the periodic domain along each axis
// (percolate), from a labelling of the whole domain and, per axis j, one with
// the periodic connection across j cut.  Cut across j, a component's pieces
// (cut components) are joined only by the boundary-crossing pairs; give each
// piece a potential, the number of periods its copy is shifted along j, with
// every crossing from coordinate n_j - 1 to 0 demanding +1.  A set of pieces
// whose crossings cannot all be satisfied contains a closed path with nonzero
// winding along j: its component percolates along j.
struct WindingSets {
    std::vector<int64_t> par, pot;  // pot[x] = potential(x) - potential(par[x])
    std::vector<char> bad;
    explicit WindingSets(size_t n) : par(n), pot(n, 0), bad(n, 0)
    {
        for (size_t i = 0; i < n; ++i) par[i] = (int64_t)i;
    }
    int64_t find(int64_t x, int64_t *px)
    {
        int64_t r = x, acc = 0;
        while (par[r] != r) {
            acc += pot[r];
            r = par[r];
        }
        int64_t y = x, accy = acc;
        while (par[y] != y) {  // compress, keeping potentials relative to the root
            const int64_t next = par[y], py = pot[y];
            par[y] = r;
            pot[y] = accy;
            accy -= py;
            y = next;
        }
        *px = acc;
        return r;
    }
    void cross(int64_t a, int64_t b)  // potential(b) = potential(a) + 1
    {
        int64_t pa, pb;
        const int64_t ra = find(a, &pa), rb = find(b, &pb);
        if (ra == rb) {
            if (pb - pa != 1) bad[ra] = 1;
        } else {
            par[rb] = ra;
            pot[rb] = pa + 1 - pb;
            bad[ra] = (char)(bad[ra] | bad[rb]);
        }
    }
};

// Flow flags of a mask's pore space: flow[t] bit j set for a pore voxel whose
// component winds along j; labels (device, N, may be null) receive the
// component labels; info (host) the counts.  flow is required.
pm_status pore_flow(pm_ctx *ctx, hipStream_t s, const uint8_t *mask, int nx, int ny, int nz, int64_t *labels,
                    uint8_t *flow, pm_pore_info *info)
{
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t dims[3] = {nx, ny, nz};
    Scratch scratch(ctx);
    void *p = nullptr;
    int64_t *lab = labels;
    if (!lab) {
        PM_TRY(scratch.get((size_t)N * sizeof(int64_t), &p));
        lab = (int64_t *)p;
    }
    int64_t max_cells = 0;
    for (int j = 0; j < 3; ++j) max_cells = std::max(max_cells, N / dims[j]);
    int64_t *cut = nullptr, *pairs = nullptr, *dlist = nullptr, *dout = nullptr;
    uint8_t *lflag = nullptr;
    unsigned long long *counts = nullptr;
    PM_TRY(scratch.get((size_t)N * sizeof(int64_t), &p));
    cut = (int64_t *)p;
    PM_TRY(scratch.get((size_t)max_cells * 2 * sizeof(int64_t), &p));
    pairs = (int64_t *)p;
    PM_TRY(scratch.get((size_t)N, &p));
    lflag = (uint8_t *)p;
    PM_TRY(scratch.get(5 * sizeof(unsigned long long), &p));
    counts = (unsigned long long *)p;
    PM_HIP(hipMemsetAsync(lflag, 0, (size_t)N, s));
    int *changed = nullptr;
    PM_TRY(scratch.get(sizeof(int), &p));
    changed = (int *)p;
    // label, then jump until every label is a root (one round when the labelling settled)
    auto label = [&](int cut_axis, int64_t *out) -> pm_status {
        PM_HIP(launch_cc_label(mask, nx, ny, nz, cut_axis, out, s));
        for (int round = 0;; ++round) {
            if (round == 64) return fail(ctx, PM_ERR_DEVICE, "pore labelling did not settle");
            int h = 0;
            PM_HIP(launch_cc_jump(out, N, changed, s));
            PM_HIP(hipMemcpyAsync(&h, changed, sizeof h, hipMemcpyDeviceToHost, s));
            PM_HIP(hipStreamSynchronize(s));
            if (!h) return PM_OK;
        }
    };
    PM_TRY(label(-1, lab));
    std::memset(info, 0, sizeof *info);
    std::vector<int64_t> hp((size_t)max_cells * 2);
    for (int j = 0; j < 3; ++j) {
        const int64_t cells = N / dims[j];
        PM_TRY(label(j, cut));
        PM_HIP(launch_cc_cross(mask, nx, ny, nz, j, cut, pairs, s));
        PM_HIP(hipMemcpyAsync(hp.data(), pairs, (size_t)cells * 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        PM_HIP(hipStreamSynchronize(s));
        // distinct crossing pairs, then the cut components they mention, densely numbered
        std::vector<std::pair<int64_t, int64_t>> pr;
        pr.reserve((size_t)cells);
        for (int64_t i = 0; i < cells; ++i)
            if (hp[2 * i] >= 0) pr.emplace_back(hp[2 * i], hp[2 * i + 1]);
        std::sort(pr.begin(), pr.end());
        pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
        std::vector<int64_t> ids;
        ids.reserve(2 * pr.size());
        for (auto &e : pr) {
            ids.push_back(e.first);
            ids.push_back(e.second);
        }
        std::sort(ids.begin(), ids.end());
        ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
        auto dense = [&](int64_t l) { return (int64_t)(std::lower_bound(ids.begin(), ids.end(), l) - ids.begin()); };
        WindingSets ws(ids.size());
        for (auto &e : pr) ws.cross(dense(e.first), dense(e.second));
        // one cut component of every winding set: its whole-domain label is the component's
        std::vector<int64_t> reps;
        for (size_t i = 0; i < ids.size(); ++i) {
            int64_t pot;
            const int64_t r = ws.find((int64_t)i, &pot);
            if (r == (int64_t)i && ws.bad[r]) reps.push_back(ids[i]);
        }
        std::vector<int64_t> plabs(reps.size());
        if (!reps.empty()) {
            Scratch lists(ctx);
            PM_TRY(lists.get(reps.size() * sizeof(int64_t), &p));
            dlist = (int64_t *)p;
            PM_TRY(lists.get(reps.size() * sizeof(int64_t), &p));
            dout = (int64_t *)p;
            PM_HIP(hipMemcpyAsync(dlist, reps.data(), reps.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
            PM_HIP(launch_gather_i64(lab, dlist, (int64_t)reps.size(), dout, s));
            PM_HIP(hipMemcpyAsync(plabs.data(), dout, reps.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            PM_HIP(hipStreamSynchronize(s));
            std::sort(plabs.begin(), plabs.end());
            plabs.erase(std::unique(plabs.begin(), plabs.end()), plabs.end());
            PM_HIP(hipMemcpyAsync(dlist, plabs.data(), plabs.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
            PM_HIP(launch_flag_labels(dlist, (int64_t)plabs.size(), j, lflag, s));
            PM_HIP(hipStreamSynchronize(s));  // the list buffers are freed at the end of this scope
        }
        info->percolates[j] = plabs.empty() ? 0 : 1;
        info->n_flowing_components[j] = (int64_t)plabs.size();
    }
    PM_HIP(launch_flow_bits(lab, lflag, N, flow, s));
    PM_HIP(launch_pore_counts(lab, flow, N, counts, s));
    unsigned long long hc[5];
    PM_HIP(hipMemcpyAsync(hc, counts, sizeof hc, hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    info->n_pore = (int64_t)hc[0];
    info->n_components = (int64_t)hc[1];
    for (int j = 0; j < 3; ++j) info->n_flowing[j] = (int64_t)hc[2 + j];
    return PM_OK;
}

}  // namespace

// ====================================================================== ABI

namespace {

// The sweeps of pm_iterate on buffers the caller of this routine provides:
// codes (N packed uint16), second (4 N values of the precision), tab (2 InstDev).
// timed: record HIP events around the sweeps into ctx->stats.  Every buffer
// is written before it is read: the codes by the preprocessing kernel, the
// second set by the first sweep launch, the table by its store kernel.
pm_status iterate_on(pm_ctx *ctx, hipStream_t s, const uint8_t *mask, int nx, int ny, int nz, int axis,
                     const pm_params *params, void *const f[4], int64_t count, void *codes, void *second,
                     InstDev *tab, bool timed)
{
    const Prec prec = params->precision == PM_FP64 ? kF64 : kF32;
    const int64_t N = (int64_t)nx * ny * nz;
    PM_HIP(launch_face_codes16(mask, nx, ny, nz, (uint16_t *)codes, s));
    PM_HIP(launch_zero_solid(prec, (const uint16_t *)codes, N, f[0], f[1], f[2], s));
    void *set[2][4];
    for (int k = 0; k < 4; ++k) {
        set[0][k] = f[k];
        set[1][k] = (char *)second + (size_t)k * N * elem(prec);
    }
    const double nu = 1.0 / params->re, c2dt = params->c2 * params->dt;
    if (params->kernel == PM_KERNEL_SIMPLE) {
        if (timed) PM_TRY(stats_mark(ctx, s, true));
        for (int64_t n = 0; n < count; ++n) {
            const int a = (int)(n & 1);
            PM_HIP(launch_simple_sweep(prec, nx, ny, nz, axis, (const uint16_t *)codes, set[a], set[a ^ 1], nu,
                                       params->dt, c2dt, params->drive, params->fixed_pressure, s));
        }
        if (timed) PM_TRY(stats_mark(ctx, s, false, 2 * count, count * N));
        if (count & 1)
            for (int k = 0; k < 4; ++k)
                PM_HIP(hipMemcpyAsync(f[k], set[1][k], (size_t)N * elem(prec), hipMemcpyDeviceToDevice, s));
        return PM_OK;
    }
    // fused: K_0 (pressure passthrough), then `count` steps; the state after
    // them is v^count (the last launch's input set) and p^count (its output).
    // With the two-step kernel, (count - 1) / 2 two-step launches come first,
    // then single steps, so that the last launch is a single step.  Launch j
    // reads set j & 1 whether it advances one sweep or two.
    Inst in;
    in.nx = nx;
    in.ny = ny;
    in.nz = nz;
    in.axis = axis;
    in.N = N;
    in.codes = (uint16_t *)codes;
    in.prec = prec;
    for (int k = 0; k < 4; ++k) {
        in.set[0][k] = set[0][k];
        in.set[1][k] = set[1][k];
    }
    in.tile = pick_tiles(ctx, params, in.nx, in.ny, in.nz, prec);
    in.nblocks = blocks_of(in);
    in.nblocks2 = blocks2_of(in);
    in.partials = nullptr;  // launches without the reduction never touch it
    const bool two = two_step(in);
    const int64_t n2 = two ? (count - 1) / 2 : 0, n1 = count - 2 * n2;
    InstDev d[3] = {make_dev(in, params, 0, true), make_dev(in, params, 0, false),
                    make_dev(in, params, 0, false, true)};
    PM_HIP(launch_store_insts(d, 3, tab, s));
    if (timed) {
        PM_TRY(ensure_events(ctx));
        PM_HIP(hipEventRecord(ctx->ev[0], s));
    }
    const bool alone = alone_of(in);
    int64_t j = 0;
    PM_HIP(launch_fused(prec, in.tile.tx, in.tile.ty, tab, 1, in.nblocks, 0, 0, s, alone));
    ++j;
    if (timed) PM_HIP(hipEventRecord(ctx->ev[2], s));
    for (int64_t k = 0; k < n2; ++k, ++j)
        PM_HIP(launch_fused2(prec, in.tile.ox, in.tile.oy, tab + 2, 1, in.nblocks2, (int)(j & 1), s));
    if (timed) PM_HIP(hipEventRecord(ctx->ev[3], s));
    for (int64_t k = 0; k < n1; ++k, ++j)
        PM_HIP(launch_fused(prec, in.tile.tx, in.tile.ty, tab + 1, 1, in.nblocks, (int)(j & 1), 0, s, alone));
    if (timed) {
        PM_HIP(hipEventRecord(ctx->ev[1], s));
        PM_HIP(hipEventSynchronize(ctx->ev[1]));
        float ms = 0.f, ms2 = 0.f;
        PM_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
        PM_HIP(hipEventElapsedTime(&ms2, ctx->ev[2], ctx->ev[3]));
        ctx->stats.sweep_ms += ms;
        ctx->stats.sweep_launches += j;
        ctx->stats.voxel_updates += (count + 1) * N;
        ctx->stats.t2_launches += n2;
        ctx->stats.t2_voxels += n2 * N;
        ctx->stats.t2_ms += n2 ? ms2 : 0.0;
        ctx->stats.tile_x = in.tile.tx;
        ctx->stats.tile_y = in.tile.ty;
        ctx->stats.zchunk = in.tile.zc;
        ctx->stats.precision = prec == kF64 ? PM_FP64 : PM_FP32;
        ctx->stats.tblock = two ? 2 : 1;
    }
    // launch j - 1 was the last: v^count in set (j - 1) & 1, p^count in set j & 1
    const int vs = (int)((j - 1) & 1), ps_ = (int)(j & 1);
    if (vs)
        for (int k = 0; k < 3; ++k)
            PM_HIP(hipMemcpyAsync(f[k], set[1][k], (size_t)N * elem(prec), hipMemcpyDeviceToDevice, s));
    if (ps_) PM_HIP(hipMemcpyAsync(f[3], set[1][3], (size_t)N * elem(prec), hipMemcpyDeviceToDevice, s));
    return PM_OK;
}

pm_status check_iterate_args(pm_ctx *ctx, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz, int axis,
                             const pm_params *params, void *const f[4], int64_t count)
{
    PM_TRY(check_params(ctx, params));
    if (params->precision == PM_FP32_DC) return fail(ctx, PM_ERR_ARG, "pm_iterate takes PM_FP64 or PM_FP32");
    if (params->outer_walls)
        return fail(ctx, PM_ERR_ARG, "outer_walls applies to solves (pm_solve, pm_tensor, pm_solve_batch)");
    const Prec prec = params->precision == PM_FP64 ? kF64 : kF32;
    PM_TRY(check_instance_args(ctx, mask, nx, ny, nz, axis, 1.0, 1.0, f, true, elem(prec)));
    if (count < 0) return fail(ctx, PM_ERR_ARG, "count must be >= 0");
    return PM_OK;
}

}  // namespace

// ------------------------------------------------------------ no allocation
//
// pm_iterate_static runs pm_iterate's sweeps on device memory that exists
// from the moment the library's code object is loaded on a GPU: one array
// per GPU, shared by every call on it.  Host code never uses the array's
// name as a device address; pm_create looks the address up once per device.
static __device__ __align__(256) unsigned char scratch[PM_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};

// Address of this device's array (the device is current); once per device.
pm_status static_scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return PM_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_ptr[dev]) return PM_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return PM_ERR_DEVICE;
    }
    g_static_ptr[dev] = ptr;
    return PM_OK;
}

void *static_scratch(int dev)
{
    std::lock_guard<std::mutex> lk(g_static_mu);
    return (dev >= 0 && dev < kMaxDevices) ? g_static_ptr[dev] : nullptr;
}

// Layout in the array: the instance table, the codes, the second field set.
constexpr size_t kStaticTab = 1024;
static_assert(4 * sizeof(InstDev) <= kStaticTab, "instance table region too small");
size_t static_bytes_needed(int64_t N, size_t e)
{
    const size_t codes = ((size_t)N * 2 + 255) / 256 * 256;
    return kStaticTab + codes + 4 * (size_t)N * e;
}

}  // namespace

extern "C" {

void pm_params_default(pm_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->re = 0.01;
    p->c2 = 1.5e6;
    p->dt = 1.0 / 4096.0;
    p->tol = 1e-8;
    p->drive = 1.0;
    p->max_sweeps = 10000000;
    p->check_every = 100;
    p->precision = PM_FP64;
    p->stop_rule = 0;
    p->warm_start = 0;
    p->kernel = PM_KERNEL_AUTO;
    p->graphs = 1;
}

const char *pm_status_string(pm_status s)
{
    switch (s) {
    case PM_OK: return "PM_OK";
    case PM_ERR_ARG: return "PM_ERR_ARG";
    case PM_ERR_OOM: return "PM_ERR_OOM";
    case PM_ERR_DEVICE: return "PM_ERR_DEVICE";
    case PM_NOT_CONVERGED: return "PM_NOT_CONVERGED";
    case PM_DIVERGED: return "PM_DIVERGED";
    case PM_ERR_NO_FLOW: return "PM_ERR_NO_FLOW";
    }
    return "PM_UNKNOWN";
}

pm_status pm_create(int hip_device, size_t mem_cap_bytes, pm_ctx **out)
{
    if (!out) return PM_ERR_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
        (void)hipGetLastError();
        return hip_device < 0 ? PM_ERR_ARG : PM_ERR_DEVICE;
    }
    pm_ctx *ctx = new (std::nothrow) pm_ctx();
    if (!ctx) return PM_ERR_OOM;
    ctx->dev = hip_device;
    ctx->cap = mem_cap_bytes;
    load_tune_cache(ctx);
    if (hipSetDevice(hip_device) != hipSuccess || static_scratch_setup(hip_device) != PM_OK) {
        (void)hipGetLastError();
        delete ctx;
        return PM_ERR_DEVICE;
    }
    *out = ctx;
    return PM_OK;
}

pm_status pm_mirror(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz, int axes,
                    uint8_t *out)
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    if (!mask || !out) return fail(ctx, PM_ERR_ARG, "mask and out must not be NULL");
    if (axes < 0 || axes > 7) return fail(ctx, PM_ERR_ARG, "axes must be a bit mask 0..7");
    PM_TRY(check_dims(ctx, nx, ny, nz));
    PM_TRY(check_dims(ctx, (axes & 1) ? 2 * nx : nx, (axes & 2) ? 2 * ny : ny, (axes & 4) ? 2 * nz : nz));
    PM_TRY(set_device(ctx));
    PM_HIP(launch_mirror(mask, (int)nx, (int)ny, (int)nz, axes, out, (hipStream_t)stream));
    return PM_OK;
}

pm_status pm_pores(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                   int64_t *labels, uint8_t *flow, pm_pore_info *info)
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    if (!mask || !info) return fail(ctx, PM_ERR_ARG, "mask and info must not be NULL");
    PM_TRY(check_dims(ctx, nx, ny, nz));
    if (labels && !aligned(labels, 8)) return fail(ctx, PM_ERR_ARG, "labels is misaligned");
    PM_TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    Scratch scratch(ctx);
    uint8_t *fl = flow;
    if (!fl) {
        void *p = nullptr;
        PM_TRY(scratch.get((size_t)(nx * ny * nz), &p));
        fl = (uint8_t *)p;
    }
    PM_TRY(pore_flow(ctx, s, mask, (int)nx, (int)ny, (int)nz, labels, fl, info));
    PM_HIP(hipStreamSynchronize(s));
    return PM_OK;
}

pm_status pm_last_stats(const pm_ctx *ctx, pm_stats *out)
{
    if (!ctx || !out) return PM_ERR_ARG;
    *out = ctx->stats;
    return PM_OK;
}

void pm_destroy(pm_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->dev);
    for (int i = 0; i < 4; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    if (ctx->d_bar) (void)hipFree(ctx->d_bar);
    if (ctx->d_fail) (void)hipFree(ctx->d_fail);
    for (auto &kv : ctx->allocs) (void)hipFree(kv.first);
    release_pool(ctx);
    if (ctx->h_sums) (void)hipHostFree(ctx->h_sums);
    delete ctx;
}

const char *pm_last_error(const pm_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

size_t pm_mem_used(const pm_ctx *ctx) { return ctx ? ctx->used + ctx->pooled : 0; }

pm_status pm_trim(pm_ctx *ctx)
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    PM_TRY(set_device(ctx));
    release_pool(ctx);
    return PM_OK;
}

pm_status pm_preprocess(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                        uint32_t *bits)
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    if (!mask || !bits) return fail(ctx, PM_ERR_ARG, "mask and bits must not be NULL");
    PM_TRY(check_dims(ctx, nx, ny, nz));
    if (!aligned(bits, 4)) return fail(ctx, PM_ERR_ARG, "bits is misaligned");
    PM_TRY(set_device(ctx));
    PM_HIP(launch_face_bits(mask, (int)nx, (int)ny, (int)nz, bits, (hipStream_t)stream));
    return PM_OK;
}

pm_status pm_face_codes(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                        uint32_t *codes)
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    if (!mask || !codes) return fail(ctx, PM_ERR_ARG, "mask and codes must not be NULL");
    PM_TRY(check_dims(ctx, nx, ny, nz));
    if (!aligned(codes, 4)) return fail(ctx, PM_ERR_ARG, "codes is misaligned");
    PM_TRY(set_device(ctx));
    PM_HIP(launch_face_codes(mask, (int)nx, (int)ny, (int)nz, codes, (hipStream_t)stream));
    return PM_OK;
}

pm_status pm_iterate(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz, int axis,
                     const pm_params *params, void *u, void *v, void *w, void *p, int64_t count)
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    void *f[4] = {u, v, w, p};
    PM_TRY(check_iterate_args(ctx, mask, nx, ny, nz, axis, params, f, count));
    PM_TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    stats_begin(ctx);
    if (count == 0) return PM_OK;
    const Prec prec = params->precision == PM_FP64 ? kF64 : kF32;
    const int64_t N = nx * ny * nz;
    Scratch scratch(ctx);
    void *codes = nullptr, *second = nullptr, *tab = nullptr;
    PM_TRY(scratch.get((size_t)N * 2, &codes));
    PM_TRY(scratch.get(4 * (size_t)N * elem(prec), &second));
    PM_TRY(scratch.get(3 * sizeof(InstDev), &tab));
    PM_TRY(iterate_on(ctx, s, mask, (int)nx, (int)ny, (int)nz, axis, params, f, count, codes, second,
                      (InstDev *)tab, true));
    // the scratch buffers are freed on return: finish the work that reads them
    PM_HIP(hipStreamSynchronize(s));
    stats_end(ctx);
    return PM_OK;
}

pm_status pm_iterate_static(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                            int axis, const pm_params *params, void *u, void *v, void *w, void *p, int64_t count)
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    void *f[4] = {u, v, w, p};
    PM_TRY(check_iterate_args(ctx, mask, nx, ny, nz, axis, params, f, count));
    const Prec prec = params->precision == PM_FP64 ? kF64 : kF32;
    const int64_t N = nx * ny * nz;
    const size_t need = static_bytes_needed(N, elem(prec));
    if (need > (size_t)PM_STATIC_SCRATCH_BYTES)
        return fail(ctx, PM_ERR_ARG,
                    "pm_iterate_static: %lld voxels need %zu bytes of static scratch, more than its %zu "
                    "(at most about %lld voxels in this precision); use pm_iterate",
                    (long long)N, need, (size_t)PM_STATIC_SCRATCH_BYTES,
                    (long long)(((size_t)PM_STATIC_SCRATCH_BYTES - kStaticTab - 256) / (4 + 4 * elem(prec))));
    PM_TRY(set_device(ctx));
    char *base = (char *)static_scratch(ctx->dev);
    if (!base) return fail(ctx, PM_ERR_DEVICE, "static scratch of device %d was not set up", ctx->dev);
    std::memset(&ctx->stats, 0, sizeof ctx->stats);
    if (count == 0) return PM_OK;
    InstDev *tab = (InstDev *)base;
    void *codes = base + kStaticTab;
    void *second = base + kStaticTab + ((size_t)N * 2 + 255) / 256 * 256;
    PM_TRY(iterate_on(ctx, (hipStream_t)stream, mask, (int)nx, (int)ny, (int)nz, axis, params, f, count, codes,
                      second, tab, false));
    PM_HIP(hipStreamSynchronize((hipStream_t)stream));
    return PM_OK;
}

pm_status pm_residual(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz, int axis,
                      const pm_params *params, const void *u, const void *v, const void *w, const void *p,
                      double out[5])
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    PM_TRY(check_params(ctx, params));
    if (params->precision == PM_FP32_DC) return fail(ctx, PM_ERR_ARG, "pm_residual takes PM_FP64 or PM_FP32");
    if (params->outer_walls) return fail(ctx, PM_ERR_ARG, "outer_walls applies to solves (pm_solve, pm_tensor, pm_solve_batch)");
    if (!out) return fail(ctx, PM_ERR_ARG, "out is NULL");
    const Prec prec = params->precision == PM_FP64 ? kF64 : kF32;
    void *f[4] = {(void *)u, (void *)v, (void *)w, (void *)p};
    PM_TRY(check_instance_args(ctx, mask, nx, ny, nz, axis, 1.0, 1.0, f, true, elem(prec)));
    PM_TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    const int64_t N = nx * ny * nz;
    Scratch scratch(ctx);
    void *codes = nullptr, *part = nullptr, *refs = nullptr, *sums = nullptr;
    PM_TRY(scratch.get((size_t)N * 2, &codes));
    PM_TRY(scratch.get((size_t)state_sums_blocks(N) * kNumSums * sizeof(double), &part));
    PM_TRY(scratch.get(sizeof(PartialRef), &refs));
    PM_TRY(scratch.get(kNumSums * sizeof(double), &sums));
    PM_HIP(launch_face_codes16(mask, (int)nx, (int)ny, (int)nz, (uint16_t *)codes, s));
    int64_t nb = 0;
    PM_HIP(launch_state_sums(prec, (int)nx, (int)ny, (int)nz, axis, (const uint16_t *)codes, f, 1.0 / params->re,
                             params->drive, params->fixed_pressure, (double *)part, &nb, s));
    PartialRef r{(const double *)part, nb};
    PM_HIP(hipMemcpyAsync(refs, &r, sizeof r, hipMemcpyHostToDevice, s));
    PM_HIP(launch_reduce_partials((const PartialRef *)refs, 1, (double *)sums, s));
    PM_HIP(hipMemcpyAsync(out, sums, kNumSums * sizeof(double), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    return PM_OK;
}

pm_status pm_autotune(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                      int precision, int32_t best[7])
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    if (!mask) return fail(ctx, PM_ERR_ARG, "mask is NULL");
    PM_TRY(check_dims(ctx, nx, ny, nz));
    if (precision != PM_FP64 && precision != PM_FP32)
        return fail(ctx, PM_ERR_ARG, "pm_autotune takes PM_FP64 or PM_FP32");
    PM_TRY(set_device(ctx));
    TileCfg c;
    PM_TRY(autotune_shape(ctx, (hipStream_t)stream, mask, (int)nx, (int)ny, (int)nz,
                          precision == PM_FP64 ? kF64 : kF32, &c));
    if (best) {
        best[0] = c.tx;
        best[1] = c.ty;
        best[2] = c.zc;
        best[3] = c.tb;
        best[4] = c.ox;
        best[5] = c.oy;
        best[6] = c.zc2;
    }
    return PM_OK;
}

pm_status pm_solve_batch(pm_ctx *ctx, void *stream, pm_instance *insts, int32_t n, const pm_params *params)
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    PM_TRY(check_params(ctx, params));
    if (!insts || n < 1) return fail(ctx, PM_ERR_ARG, "need at least one instance");
    if (params->kernel == PM_KERNEL_SIMPLE)
        return fail(ctx, PM_ERR_ARG, "solves use the fused kernel (PM_KERNEL_SIMPLE is for pm_iterate)");
    const size_t align = params->precision == PM_FP32 ? sizeof(float) : sizeof(double);
    std::vector<Inst> list((size_t)n);
    for (int i = 0; i < n; ++i) {
        pm_instance &pi = insts[i];
        void *f[4] = {pi.u, pi.v, pi.w, pi.p};
        pm_status s = check_instance_args(ctx, pi.mask, pi.nx, pi.ny, pi.nz, pi.axis, pi.voxel_size, pi.mu, f,
                                          false, align);
        if (s != PM_OK) {
            ctx->err = "instance " + std::to_string(i) + ": " + ctx->err;
            return s;
        }
        if (params->warm_start && !pi.u)
            return fail(ctx, PM_ERR_ARG, "instance %d: warm_start needs field pointers", i);
        Inst &in = list[i];
        in.mask = pi.mask;
        in.nx = (int)pi.nx;
        in.ny = (int)pi.ny;
        in.nz = (int)pi.nz;
        in.N = pi.nx * pi.ny * pi.nz;
        in.axis = pi.axis;
        in.dx = pi.voxel_size;
        in.mu = pi.mu;
        for (int k = 0; k < 4; ++k) in.user[k] = f[k];
        in.hist = pi.hist;
        if (in.hist) in.hist->n = 0;
    }
    PM_TRY(set_device(ctx));
    stats_begin(ctx);
    // outer walls: sweep each instance on its grid with one solid layer appended
    // along every wall axis; the fields come back to the caller's grid afterwards
    struct Walled {
        int nx = 0, ny = 0, nz = 0;
        int64_t N = 0;
        void *user[4] = {nullptr, nullptr, nullptr, nullptr};
    };
    std::vector<Walled> walled(list.size());
    Scratch wall_scratch(ctx);
    const int W = params->outer_walls;
    const size_t wall_ue = params->precision == PM_FP32 ? sizeof(float) : sizeof(double);
    if (W) {
        std::map<const uint8_t *, const uint8_t *> padded_of;
        for (size_t i = 0; i < list.size(); ++i) {
            Inst &in = list[i];
            Walled &w = walled[i];
            w.nx = in.nx;
            w.ny = in.ny;
            w.nz = in.nz;
            w.N = in.N;
            for (int f = 0; f < 4; ++f) w.user[f] = in.user[f];
            const int px = in.nx + (W & 1), py = in.ny + ((W >> 1) & 1), pz = in.nz + ((W >> 2) & 1);
            PM_TRY(check_dims(ctx, px, py, pz));
            const int64_t Np = (int64_t)px * py * pz;
            void *p = nullptr;
            auto it = padded_of.find(in.mask);
            if (it != padded_of.end()) {
                in.mask = it->second;
            } else {
                PM_TRY(wall_scratch.get((size_t)Np, &p));
                PM_HIP(launch_pad_mask(in.mask, in.nx, in.ny, in.nz, (uint8_t *)p, px, py, pz, (hipStream_t)stream));
                padded_of[in.mask] = (const uint8_t *)p;
                in.mask = (const uint8_t *)p;
            }
            PM_TRY(wall_scratch.get(4 * (size_t)Np * wall_ue, &p));
            for (int f = 0; f < 4; ++f) {
                void *pf = (char *)p + (size_t)f * Np * wall_ue;
                if (params->warm_start)
                    PM_HIP(launch_embed(wall_ue, w.user[f], in.nx, in.ny, in.nz, pf, px, py, pz, (hipStream_t)stream));
                else
                    PM_HIP(hipMemsetAsync(pf, 0, (size_t)Np * wall_ue, (hipStream_t)stream));
                in.user[f] = pf;
            }
            in.nx = px;
            in.ny = py;
            in.nz = pz;
            in.N = Np;
            in.no_through_flow = (W >> in.axis) & 1;
        }
    }
    // pore cleanup: each instance sweeps a copy of its mask in which the pore
    // components that do not wind along its load axis are solid
    Scratch cleaned(ctx);
    if (params->pore_cleanup) {
        std::map<const uint8_t *, uint8_t *> flow_of;
        for (Inst &in : list) {
            uint8_t *flow = nullptr;
            auto it = flow_of.find(in.mask);
            if (it != flow_of.end()) {
                flow = it->second;
            } else {
                void *p = nullptr;
                PM_TRY(cleaned.get((size_t)in.N, &p));
                flow = (uint8_t *)p;
                pm_pore_info info;
                PM_TRY(pore_flow(ctx, (hipStream_t)stream, in.mask, in.nx, in.ny, in.nz, nullptr, flow, &info));
                flow_of[in.mask] = flow;
            }
            void *p = nullptr;
            PM_TRY(cleaned.get((size_t)in.N, &p));
            PM_HIP(launch_clean_mask(flow, in.N, in.axis, (uint8_t *)p, (hipStream_t)stream));
            in.mask = (const uint8_t *)p;
        }
    }
    if (params->autotune && !(params->tile_x && params->tile_y) && params->zchunk == 0) {
        std::vector<Prec> precs;
        if (params->precision != PM_FP64) precs.push_back(kF32);
        if (params->precision != PM_FP32) precs.push_back(kF64);
        for (const Inst &in : list)
            for (Prec pr : precs)
                if (!ctx->tune.count(tune_key(in.nx, in.ny, in.nz, pr)))
                    PM_TRY(autotune_shape(ctx, (hipStream_t)stream, in.mask, in.nx, in.ny, in.nz, pr, nullptr));
    }
    pm_status rs;
    {
        Engine eng(ctx, (hipStream_t)stream, params, list);
        rs = eng.run();
    }
    if (W && rs == PM_OK) {
        // back to the caller's grid: fields (solved instances), and the flux and k
        // as means over the caller's voxels
        for (size_t i = 0; i < list.size(); ++i) {
            Inst &in = list[i];
            const Walled &w = walled[i];
            if (in.status != PM_ERR_NO_FLOW && w.user[0])
                for (int f = 0; f < 4; ++f)
                    PM_HIP(launch_extract(wall_ue, in.user[f], in.nx, in.ny, w.user[f], w.nx, w.ny, w.nz,
                                          (hipStream_t)stream));
            const double sc = (double)in.N / (double)w.N;
            for (int k = 0; k < 3; ++k) in.kcol[k] *= sc;
            if (in.hist && in.hist->q)
                for (int64_t j = 0; j < in.hist->n; ++j)
                    for (int k = 0; k < 3; ++k) in.hist->q[3 * j + k] *= sc;
        }
        PM_HIP(hipStreamSynchronize((hipStream_t)stream));
    }
    stats_end(ctx);
    pm_status worst = PM_OK;
    for (int i = 0; i < n; ++i) {
        pm_instance &pi = insts[i];
        const Inst &in = list[i];
        pi.status = rs != PM_OK ? rs : in.status;
        pi.sweeps = in.sweeps;
        for (int k = 0; k < 3; ++k) pi.k_col[k] = in.kcol[k];
        if (severity((pm_status)pi.status) > severity(worst)) worst = (pm_status)pi.status;
    }
    return rs != PM_OK ? rs : worst;
}

pm_status pm_solve(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                   double voxel_size, double mu, int axis, const pm_params *params, void *u, void *v, void *w,
                   void *p, pm_history *hist, double k_col[3], int64_t *sweeps_done)
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    if (!k_col) return fail(ctx, PM_ERR_ARG, "k_col is NULL");
    if (!u || !v || !w || !p) return fail(ctx, PM_ERR_ARG, "field pointers must not be NULL");
    pm_instance in;
    std::memset(&in, 0, sizeof in);
    in.mask = mask;
    in.nx = nx;
    in.ny = ny;
    in.nz = nz;
    in.voxel_size = voxel_size;
    in.mu = mu;
    in.axis = axis;
    in.u = u;
    in.v = v;
    in.w = w;
    in.p = p;
    in.hist = hist;
    pm_status s = pm_solve_batch(ctx, stream, &in, 1, params);
    for (int k = 0; k < 3; ++k) k_col[k] = in.k_col[k];
    if (sweeps_done) *sweeps_done = in.sweeps;
    return s;
}

pm_status pm_tensor(pm_ctx *ctx, void *stream, const uint8_t *mask, int64_t nx, int64_t ny, int64_t nz,
                    double voxel_size, double mu, const pm_params *params, double k[9], double k_sym[9],
                    pm_history *hist, int64_t sweeps[3])
{
    if (!ctx) return PM_ERR_ARG;
    ctx->err.clear();
    if (!k || !k_sym) return fail(ctx, PM_ERR_ARG, "k and k_sym must not be NULL");
    pm_instance in[3];
    std::memset(in, 0, sizeof in);
    for (int j = 0; j < 3; ++j) {
        in[j].mask = mask;
        in[j].nx = nx;
        in[j].ny = ny;
        in[j].nz = nz;
        in[j].voxel_size = voxel_size;
        in[j].mu = mu;
        in[j].axis = j;
        in[j].hist = hist ? &hist[j] : nullptr;
    }
    PM_TRY(check_params(ctx, params));
    if (params->warm_start) return fail(ctx, PM_ERR_ARG, "pm_tensor keeps its fields internally");
    PM_TRY(check_dims(ctx, nx, ny, nz));
    PM_TRY(set_device(ctx));
    // The three load cases run as one batch when their buffers fit beside each
    // other (the context cap and the device's free memory, kept blocks counted
    // as free), else one after another: each solve's iterate is the same either
    // way (an untuned batch decomposes every instance as its single solve).
    bool together = true;
    {
        const int64_t N = nx * ny * nz;
        const size_t ue = params->precision == PM_FP32 ? sizeof(float) : sizeof(double);
        // stencil codes once, per load case caller-set and internal set (and the
        // correction form's defect field), rounded up for padding by outer walls
        const size_t per_case = 8 * (size_t)N * ue + (params->precision == PM_FP32_DC ? 16 * (size_t)N : 0);
        const size_t need = (size_t)(1.02 * (double)(2 * (size_t)N + 3 * per_case));
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            free_b = SIZE_MAX / 2;
        }
        size_t avail = free_b + ctx->pooled;
        if (ctx->cap) avail = std::min(avail, ctx->cap > ctx->used ? ctx->cap - ctx->used : (size_t)0);
        together = need <= avail;
    }
    pm_status s;
    if (together) {
        s = pm_solve_batch(ctx, stream, in, 3, params);
        ctx->stats.tensor_cases_at_once = 3;
    } else {
        pm_stats sum{};
        s = PM_OK;
        for (int j = 0; j < 3; ++j) {
            const pm_status sj = pm_solve_batch(ctx, stream, &in[j], 1, params);
            const pm_stats &st = ctx->stats;
            sum.sweep_launches += st.sweep_launches;
            sum.voxel_updates += st.voxel_updates;
            sum.sweep_ms += st.sweep_ms;
            sum.total_ms += st.total_ms;
            sum.tile_x = st.tile_x;
            sum.tile_y = st.tile_y;
            sum.zchunk = st.zchunk;
            sum.precision = st.precision;
            sum.tblock = st.tblock;
            sum.peak_bytes = std::max(sum.peak_bytes, st.peak_bytes);
            sum.dc_promoted_for_memory += st.dc_promoted_for_memory;
            if (severity(sj) > severity(s)) s = sj;
            if (sj == PM_ERR_ARG || sj == PM_ERR_OOM || sj == PM_ERR_DEVICE) break;
        }
        sum.tensor_cases_at_once = 1;
        ctx->stats = sum;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) k[i * 3 + j] = in[j].k_col[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) k_sym[i * 3 + j] = 0.5 * (k[i * 3 + j] + k[j * 3 + i]);
    if (sweeps)
        for (int j = 0; j < 3; ++j) sweeps[j] = in[j].sweeps;
    return s;
}

}  // extern "C"
