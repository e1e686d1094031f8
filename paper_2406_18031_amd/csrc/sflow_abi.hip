// Host runtime and C ABI of the structure-flow filter (see include/sflow.h).
//
// A context is a batch of camera streams (one for sf_create).  It owns one device arena that
// holds, for every (stream, level) "entry", the double-buffered state planes (w, dw, rho,
// Yhat) and the level's pyramid image and inverse depth, all row-major with rows padded to
// 256 bytes, plus the entry table the kernels read.  A frame of every stream is: the pyramid
// (one launch per pyramid depth, all streams together), one fused level-step launch covering
// every tile of every level of every stream (levels are independent within a frame), then the
// coarse-to-fine reconstruction (one launch per depth, all streams together).  With the
// learned update, the network and the choice kernel run between the step and the
// reconstruction.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <stdlib.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sflow_cnn.h"
#include "sflow_internal.h"

using namespace sflow;

struct StreamInfo {
    sf_config cfg{};
    int H = 0;
    int e0 = 0;                    // first entry of the stream (its finest level)
    double cam[4] = {0, 0, 0, 0};
    double dt_prev = 0.0;
    bool update_ran = false;       // an update has run since the camera or the state was set
    bool stereo = false;           // stereo parameters for sf_stereo_depth are set
    double baseline = 0.0, texture = 0.0, residual = 0.0;
    int dmax = 0, iters = 0;
    bool source = false;           // a source camera for sf_map_frame is set
    double src[4] = {0, 0, 0, 0};  // its intrinsics
    int src_rows = 0, src_cols = 0;
};

struct sf_ctx_s {
    int S = 0;                     // streams
    // The frame's last reconstruction launch (the one holding the finest levels) waits for the
    // next call that needs them, so that sf_get_flow can run it together with the output.
    bool recon_pending = false;
    int storage = SF_FP32;
    hipStream_t stream = nullptr;
    int esize = 4;                 // bytes per stored element
    bool camera = false;
    bool hip_failed = false;
    int64_t frames = 0;            // frames pushed since the cameras were set
    int parity = 0;                // state[parity] holds the latest frame
    std::string err;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    std::vector<StreamInfo> st;
    std::vector<LevelDev> lv;      // entries, stream by stream, finest level first
    LevelDev* lv_dev = nullptr;
    int user_tw[kMaxLevels]{};
    int user_th[kMaxLevels]{};
    // step launches: the prediction of a level with N > pass_steps is split into passes
    int pass_steps = kDefaultPassSteps;
    struct StepLaunch { int e0, n, nblocks; };
    std::vector<LevelDev> sv;       // pass entries, launch by launch
    std::vector<StepLaunch> step_launches;
    LevelDev* sv_dev = nullptr;
    size_t sv_cap = 0;              // entries sv_dev can hold
    float* mid = nullptr;           // FP32 fields between passes (two sets per split level)
    float* geo = nullptr;           // geometry tables of every level (general grids), or NULL
    bool grid = false;              // the level steps read geometry tables
    bool grid_pinhole[kMaxStreams] = {};   // stream s's table holds its pinhole's own rays
    size_t mid_bytes = 0;
    size_t lds_bytes = 0;
    int max_levels = 0;
    // timing
    bool timing = false;
    struct Mark { hipEvent_t a, b; int kind; };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> pool;
    double ms[3] = {0, 0, 0};
    int64_t launches[3] = {0, 0, 0};
    // learned update (finest level of every stream)
    bool learned = false;
    bool weights = false;
    float threshold = 1.0f;
    CnnSegs segs{};
    float* lbuf = nullptr;               // kLearnPlanes x ltotal
    uint16_t* lpack = nullptr;           // the network's input, BF16 NHWC 16 (in lbuf's allocation)
    uint16_t* act[2] = {nullptr, nullptr};   // BF16 NHWC 16-channel activations
    uint16_t* wf = nullptr;              // packed forward weights [4][9][16][16]
    uint16_t* wb = nullptr;
    float* cnn_bias = nullptr;           // [4][16]
    float* params_dev = nullptr;         // FP32 master weights
    unsigned long long* fallbacks = nullptr;
    unsigned long long* numeric = nullptr;    // watchdog word (LevelDev::numeric), in the arena
    int64_t learned_pixels = 0;
    // Frame graphs (sf_set_graph): a frame's launches after the first frame, captured once per
    // state parity and per form of the prediction (plain / inertial), replayed with the
    // per-frame arguments of the pyramid and level-step nodes updated in place.
    struct FrameArgsNode {
        hipGraphNode_t node = nullptr;
        hipKernelNodeParams p{};     // launch shape and kernel of the node
        int kind = 0;                // frame_input_kind of its kernel
        ElemArgs e{};                // its arguments (kind 1)
        StepArgs st{};               // its arguments (kind 2)
    };
    struct FrameGraph {
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        std::vector<FrameArgsNode> nodes;
    };
    bool graph_on = false;
    hipStream_t cap = nullptr;            // private stream the frame is captured on
    FrameGraph graphs[2][2];              // [parity][inertial]
    // Inputs produced on a stream of the caller's (sf_set_input_stream): each push builds the
    // frame's pyramid on pyr_stream, after the work on in_stream (ev_in) and after the level
    // step that last read the pyramid buffer it writes (ev_step[buffer]); the context stream
    // waits for the pyramid (ev_pyr); the input stream waits for the previous frame's level
    // step before the push returns.
    hipStream_t in_stream = nullptr;      // NULL: inputs are ordered on the context stream
    hipStream_t pyr_stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_pyr = nullptr, ev_step[2] = {nullptr, nullptr};
    bool step_rec[2] = {false, false};    // ev_step[m] holds a frame's record
    int mbuf = 0;                         // pyramid buffer of the next frame
};

static std::string g_create_error;

// Every device allocation of the library goes through dev_malloc.  For testing the error
// paths, SFLOW_FAIL_ALLOC=n in the environment makes the n-th allocation counted from the
// moment the variable took its current value fail as if the device were out of memory.
hipError_t sflow::dev_malloc(void** p, size_t bytes) {
    static std::mutex mu;
    static std::string seen;
    static long count = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        const char* v = getenv("SFLOW_FAIL_ALLOC");
        const std::string cur = v ? v : "";
        if (cur != seen) {
            seen = cur;
            count = 0;
        }
        if (!cur.empty() && ++count == strtol(cur.c_str(), nullptr, 10)) {
            *p = nullptr;
            return hipErrorOutOfMemory;
        }
    }
    return hipMalloc(p, bytes);
}

static sf_status fail(sf_ctx c, sf_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf; else g_create_error = buf;
    return s;
}

static sf_status hip_fail(sf_ctx c, hipError_t e, const char* what) {
    if (c) c->hip_failed = true;
    return fail(c, SF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                                        \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);                  \
    } while (0)

static int level_halo(int N, int Ns) { return std::max(N, 2) + 2 * Ns; }

// A prediction of N steps split into passes of at most ps steps: the number of passes and the
// steps of pass i (equal shares, the last one taking the rest).
static int npasses(int N, int ps) { return (N + ps - 1) / ps; }
static int pass_len(int N, int P, int i) {
    const int q = (N + P - 1) / P;
    return i < P - 1 ? q : N - (P - 1) * q;
}
// halo of the last pass, the largest of the level's passes
static int last_pass_halo(int N, int Ns, int ps) {
    const int P = npasses(N, ps);
    return level_halo(pass_len(N, P, P - 1), Ns);
}

static int level_steps(float max_flow, int h) {   // h is 0-based
    double v = ceil((double)max_flow / ldexp(1.0, h));
    return std::max(1, (int)v);
}

static bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

static sf_status check_alive(sf_ctx c) {
    if (!c) return fail(nullptr, SF_ERR_INVALID_ARG, "NULL context");
    if (c->hip_failed) return fail(c, SF_ERR_HIP, "context unusable after a HIP failure: %s",
                                   c->err.c_str());
    return SF_OK;
}

static const float kDefaultAlpha[5] = {300.0f, 1000.0f, 1.0f, 1.0f, 1.0f};

static sf_status validate_config(const sf_config* cfg, sf_config* out) {
    if (!cfg) return fail(nullptr, SF_ERR_INVALID_ARG, "NULL config");
    sf_config c = *cfg;
    if (c.rows < 2 || c.cols < 2) return fail(nullptr, SF_ERR_INVALID_ARG, "rows and cols must be >= 2");
    if (c.rows > (1 << 15) || c.cols > (1 << 15))
        return fail(nullptr, SF_ERR_INVALID_ARG, "rows and cols must be <= 32768");
    if (c.levels < 1 || c.levels > kMaxLevels)
        return fail(nullptr, SF_ERR_INVALID_ARG, "levels must be in [1, %d]", kMaxLevels);
    int r = c.rows, q = c.cols;
    for (int h = 1; h < c.levels; ++h) { r = (r + 1) / 2; q = (q + 1) / 2; }
    if (r < 2 || q < 2)
        return fail(nullptr, SF_ERR_INVALID_ARG, "the coarsest level must be at least 2x2");
    if (!(c.max_flow_px >= 0.0f) || !isfinite(c.max_flow_px) || c.max_flow_px > 4096.0f)
        return fail(nullptr, SF_ERR_INVALID_ARG, "max_flow_px must be finite and in [0, 4096]");
    for (int h = 0; h < c.levels; ++h)
        if (c.smooth_iters[h] < 0 || c.smooth_iters[h] > 16)
            return fail(nullptr, SF_ERR_INVALID_ARG, "smooth_iters must be in [0, 16]");
    bool allzero = true;
    for (int k = 0; k < 5; ++k) allzero = allzero && c.alpha[k] == 0.0f;
    if (allzero) memcpy(c.alpha, kDefaultAlpha, sizeof kDefaultAlpha);
    for (int k = 0; k < 5; ++k)
        if (!(c.alpha[k] >= 0.0f) || !isfinite(c.alpha[k]))
            return fail(nullptr, SF_ERR_INVALID_ARG, "alpha must be finite and >= 0");
    if (!(c.alpha[2] > 0.0f)) return fail(nullptr, SF_ERR_INVALID_ARG, "alpha_3 must be > 0");
    if (!(c.alpha[3] + c.alpha[4] > 0.0f))
        return fail(nullptr, SF_ERR_INVALID_ARG, "alpha_4 + alpha_5 must be > 0");
    if (c.storage != SF_FP32 && c.storage != SF_FP16)
        return fail(nullptr, SF_ERR_INVALID_ARG, "storage must be SF_FP32 or SF_FP16");
    if (c.update != SF_UPDATE_PLAIN && c.update != SF_UPDATE_LEARNED)
        return fail(nullptr, SF_ERR_INVALID_ARG, "unknown update kind");
    if (c.update == SF_UPDATE_LEARNED && c.smooth_iters[0] > 4)
        return fail(nullptr, SF_ERR_UNSUPPORTED,
                    "the learned update supports at most 4 smoothing passes at the finest level");
    if (c.read_flags & ~(uint32_t)(SF_READ_DOMINANT_LITERAL | SF_READ_SOURCE_LITERAL |
                                    SF_READ_NO_CFL_CLAMP))
        return fail(nullptr, SF_ERR_INVALID_ARG, "unknown read_flags bits");
    for (int h = 0; h < c.levels; ++h) {
        int halo = last_pass_halo(level_steps(c.max_flow_px, h), c.smooth_iters[h],
                                  kDefaultPassSteps);
        if (2 * halo >= kRegion)
            return fail(nullptr, SF_ERR_UNSUPPORTED,
                        "level %d needs a halo of %d pixels (max(N,2) + 2*smooth); at most %d fit",
                        h + 1, halo, (kRegion - 1) / 2);
    }
    for (int h = c.levels; h < kMaxLevels; ++h) c.smooth_iters[h] = 0;
    *out = c;
    return SF_OK;
}

// Tiles of an entry: a balanced split of the level into tiles of at most 64 - 2*halo.
static void choose_tiles(sf_ctx c, LevelDev& L) {
    const int tmax = kRegion - 2 * L.halo;
    int tw = c->user_tw[L.level], th = c->user_th[L.level];
    if (tw <= 0 || th <= 0 || tw > tmax || th > tmax) {
        int nx = (L.cols + tmax - 1) / tmax, ny = (L.rows + tmax - 1) / tmax;
        tw = (L.cols + nx - 1) / nx;
        th = (L.rows + ny - 1) / ny;
    }
    L.tw = tw;
    L.th = th;
    L.tiles_x = (L.cols + tw - 1) / tw;
    L.tiles_y = (L.rows + th - 1) / th;
}

// Pass entries and step launches, computed into `out` from the context's levels, pass length
// and tile choices (the context itself is not changed).  A level with P passes runs pass i in
// launch Pmax - P + i, so every level's last pass (update, smoothing, store) is in the last
// launch.  `mid` is the base of the FP32 intermediate fields of split levels (NULL: not yet
// allocated; the pass entries then hold NULL for them).  Returns the bytes of those fields.
struct Layout {
    std::vector<LevelDev> lv;                       // the levels with their last pass's tiles
    std::vector<LevelDev> sv;                       // pass entries, launch by launch
    std::vector<sf_ctx_s::StepLaunch> launches;
};

static size_t layout_blocks(sf_ctx c, float* mid, Layout& out) {
    out.lv = c->lv;
    out.sv.clear();
    out.launches.clear();
    int pmax = 1;
    for (auto& L : out.lv) pmax = std::max(pmax, npasses(L.N, c->pass_steps));
    size_t mid_off = 0;
    std::vector<size_t> mid_at(out.lv.size(), 0);
    for (size_t e = 0; e < out.lv.size(); ++e) {
        const LevelDev& L = out.lv[e];
        if (npasses(L.N, c->pass_steps) > 1) {
            mid_at[e] = mid_off;
            mid_off += 2 * 8 * ((size_t)L.rows * L.pitch * sizeof(float) + 255) / 256 * 256;
        }
    }
    for (int k = 0; k < pmax; ++k) {
        sf_ctx_s::StepLaunch sl{(int)out.sv.size(), 0, 0};
        int b = 0;
        for (size_t e = 0; e < out.lv.size(); ++e) {
            LevelDev& L = out.lv[e];
            const int P = npasses(L.N, c->pass_steps);
            const int i = k - (pmax - P);
            if (i < 0) continue;
            LevelDev S = L;
            S.pass_n = pass_len(L.N, P, i);
            S.pass_first = i == 0;
            S.pass_last = i == P - 1;
            S.halo = S.pass_last ? level_halo(S.pass_n, L.Ns) : S.pass_n;
            const size_t plane = ((size_t)L.rows * L.pitch * sizeof(float) + 255) / 256 * 256;
            for (int f = 0; f < 8; ++f) {
                S.mid_in[f] = nullptr;
                S.mid_out[f] = nullptr;
                if (P > 1 && mid) {
                    float* base = (float*)((char*)mid + mid_at[e]);
                    if (!S.pass_first)
                        S.mid_in[f] = (float*)((char*)base + (((i - 1) & 1) * 8 + f) * plane);
                    if (!S.pass_last)
                        S.mid_out[f] = (float*)((char*)base + ((i & 1) * 8 + f) * plane);
                }
            }
            choose_tiles(c, S);
            S.block0 = b;
            b += S.tiles_x * S.tiles_y;
            if (S.pass_last) {   // the level's own entry keeps the tiles of its last pass
                L.tw = S.tw; L.th = S.th; L.tiles_x = S.tiles_x; L.tiles_y = S.tiles_y;
                L.halo = S.halo;
            }
            out.sv.push_back(S);
            ++sl.n;
        }
        sl.nblocks = b;
        out.launches.push_back(sl);
    }
    return mid_off;
}

// per-pixel launch over the entries of level `level` (all streams that have it)
static ElemArgs elem_args(sf_ctx c, int level, int parity) {
    ElemArgs a{};
    a.lv = c->lv_dev;
    a.parity = parity;
    int b = 0;
    for (int s = 0; s < c->S; ++s) {
        const StreamInfo& si = c->st[s];
        if (level >= si.H) continue;
        const int e = si.e0 + level;
        a.ent[a.n] = e;
        a.blk[a.n] = b;
        b += (c->lv[e].rows * c->lv[e].cols + kElemBlock - 1) / kElemBlock;
        ++a.n;
    }
    a.blk[a.n] = b;
    return a;
}

// A two-level tile launch (pyramid, reconstruction) at `level` over the streams with more than
// level + above levels.
static ElemArgs tile_args(sf_ctx c, int level, int above, int parity, int tile = kTile2) {
    ElemArgs a{};
    a.lv = c->lv_dev;
    a.parity = parity;
    int b = 0;
    for (int s = 0; s < c->S; ++s) {
        const StreamInfo& si = c->st[s];
        if (level + above >= si.H) continue;
        const int e = si.e0 + level;
        a.ent[a.n] = e;
        a.blk[a.n] = b;
        b += ((c->lv[e].rows + tile - 1) / tile) * ((c->lv[e].cols + tile - 1) / tile);
        ++a.n;
    }
    a.blk[a.n] = b;
    return a;
}

// Tile side of a pyramid (above = 0) or reconstruction (above = 1) launch over level h.  From
// kBigLaunch kTile2 tiles on (16 per CU) it is 2 kTile2: four times the pixels per block, a
// quarter of the blocks and of the re-read margins (reconstruction of a batch of 64 streams:
// 464 -> 268 us per frame).  Below that a launch is short and latency-bound and the smaller
// tile is faster (reconstruction of one 512 x 512 stream: 8.3 us against 9.8).  Both tiles
// give bitwise the same results.
static constexpr int kBigLaunch = 16 * 256;

static int big_tile(sf_ctx c, int level, int above) {
    const ElemArgs a = tile_args(c, level, above, 0);
    return a.blk[a.n] >= kBigLaunch ? 2 * kTile2 : kTile2;
}

static int recon_tile(sf_ctx c, int level) { return big_tile(c, level, 1); }

extern "C" {

static sf_status flush_recon(sf_ctx c);
static void drop_graphs(sf_ctx c);

sf_status sf_create_batch(const sf_config* cfgs, int32_t n, void* hip_stream, sf_ctx* out) {
    if (!out) return fail(nullptr, SF_ERR_INVALID_ARG, "NULL output pointer");
    *out = nullptr;
    if (!cfgs) return fail(nullptr, SF_ERR_INVALID_ARG, "NULL config");
    if (n < 1 || n > kMaxStreams)
        return fail(nullptr, SF_ERR_INVALID_ARG, "stream count must be in [1, %d]", kMaxStreams);
    std::vector<sf_config> cf(n);
    for (int s = 0; s < n; ++s) {
        sf_status st = validate_config(&cfgs[s], &cf[s]);
        if (st != SF_OK) {
            if (n > 1) g_create_error = "stream " + std::to_string(s) + ": " + g_create_error;
            return st;
        }
        if (cf[s].storage != cf[0].storage)
            return fail(nullptr, SF_ERR_INVALID_ARG, "all streams of a batch need the same storage");
        if (cf[s].update != cf[0].update)
            return fail(nullptr, SF_ERR_INVALID_ARG, "all streams of a batch need the same update");
    }
    sf_ctx ctx = new (std::nothrow) sf_ctx_s();
    if (!ctx) return fail(nullptr, SF_ERR_OOM, "host allocation failed");
    ctx->S = n;
    ctx->storage = cf[0].storage;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->esize = ctx->storage == SF_FP16 ? 2 : 4;
    ctx->st.resize(n);
    const size_t align = 256;
    auto plane_bytes = [&](int rows, int pitch) {
        return ((size_t)rows * pitch * ctx->esize + align - 1) / align * align;
    };
    size_t total = 0;
    for (int s = 0; s < n; ++s) {
        StreamInfo& si = ctx->st[s];
        si.cfg = cf[s];
        si.H = cf[s].levels;
        si.e0 = (int)ctx->lv.size();
        ctx->max_levels = std::max(ctx->max_levels, si.H);
        int r = cf[s].rows, q = cf[s].cols;
        for (int h = 0; h < si.H; ++h) {
            LevelDev L{};
            L.rows = r;
            L.cols = q;
            const int per_row = (int)(align / ctx->esize);
            L.pitch = (q + per_row - 1) / per_row * per_row;
            L.top = h == si.H - 1;
            L.stream = s;
            L.level = h;
            L.child = h > 0 ? si.e0 + h - 1 : -1;
            L.parent = h + 1 < si.H ? si.e0 + h + 1 : -1;
            L.flags = cf[s].read_flags;
            const int nplanes = 2 * (3 + (L.top ? 0 : 3) + 2) + (h > 0 ? 4 : 0);
            total += nplanes * plane_bytes(r, L.pitch);
            ctx->lv.push_back(L);
            r = (r + 1) / 2;
            q = (q + 1) / 2;
        }
    }
    total += align + sizeof(LevelDev) * (ctx->lv.size() + kLevelPad);   // zeroed padding
    total += 256;                                                          // watchdog word
    hipError_t e = dev_malloc((void**)&ctx->arena, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return fail(nullptr, e == hipErrorOutOfMemory ? SF_ERR_OOM : SF_ERR_HIP,
                    "hipMalloc of %zu bytes failed: %s", total, hipGetErrorString(e));
    }
    ctx->arena_bytes = total;
    char* p = ctx->arena;
    auto take = [&](size_t nb) { char* x = p; p += nb; return (void*)x; };
    for (auto& L : ctx->lv) {
        const size_t pb = plane_bytes(L.rows, L.pitch);
        for (int par = 0; par < 2; ++par) {
            for (int k = 0; k < 3; ++k) L.w[par][k] = take(pb);
            for (int k = 0; k < 3; ++k) L.dw[par][k] = L.top ? nullptr : take(pb);
            L.rho[par] = take(pb);
            L.Y[par] = take(pb);
        }
        for (int m = 0; m < 2; ++m) {
            L.Ym[m] = L.level > 0 ? take(pb) : nullptr;
            L.Rm[m] = L.level > 0 ? take(pb) : nullptr;
        }
    }
    ctx->lv_dev = (LevelDev*)take(sizeof(LevelDev) * (ctx->lv.size() + kLevelPad));
    ctx->numeric = (unsigned long long*)take(256);
    for (auto& L : ctx->lv) L.numeric = ctx->numeric;
    if (cf[0].update == SF_UPDATE_LEARNED) {
        ctx->learned = true;
        CnnSegs& sg = ctx->segs;
        sg.n = n;
        int b = 0;
        int o = 0;
        for (int s = 0; s < n; ++s) {
            sg.base[s] = b;
            sg.off[s] = o;
            sg.rows[s] = cf[s].rows;
            sg.cols[s] = cf[s].cols;
            b += (cf[s].rows * cf[s].cols + 15) / 16 * 16;
            o += cf[s].rows * cf[s].cols;
        }
        sg.base[n] = b;
        sg.off[n] = o;
        sg.total = b;
        size_t lb_bytes = (size_t)kLearnPlanes * b * sizeof(float);
        size_t act_bytes = (size_t)b * 16 * sizeof(uint16_t);
        size_t need = lb_bytes + 3 * act_bytes + 2 * 4 * 9 * 256 * sizeof(uint16_t) +
                      4 * 16 * sizeof(float) + kCnnParams * sizeof(float) + 64 + 6 * 256;
        hipError_t e2 = dev_malloc((void**)&ctx->lbuf, need);
        if (e2 != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(ctx->arena);
            delete ctx;
            return fail(nullptr, e2 == hipErrorOutOfMemory ? SF_ERR_OOM : SF_ERR_HIP,
                        "hipMalloc of the learned buffers failed: %s", hipGetErrorString(e2));
        }
        auto al = [](size_t v) { return (v + 255) / 256 * 256; };
        char* q = (char*)ctx->lbuf + al(lb_bytes);
        ctx->act[0] = (uint16_t*)q; q += al(act_bytes);
        ctx->act[1] = (uint16_t*)q; q += al(act_bytes);
        ctx->lpack = (uint16_t*)q; q += al(act_bytes);
        ctx->wf = (uint16_t*)q; q += al(4 * 9 * 256 * sizeof(uint16_t));
        ctx->wb = (uint16_t*)q; q += al(4 * 9 * 256 * sizeof(uint16_t));
        ctx->cnn_bias = (float*)q; q += al(4 * 16 * sizeof(float));
        ctx->params_dev = (float*)q; q += al(kCnnParams * sizeof(float));
        ctx->fallbacks = (unsigned long long*)q;
        for (int s = 0; s < n; ++s) {
            LevelDev& L = ctx->lv[ctx->st[s].e0];
            L.learned = 1;
            L.lbase = sg.base[s];
            L.ltotal = b;
            L.lbuf = ctx->lbuf;
            L.lpack = ctx->lpack;
        }
        e2 = hipMemsetAsync(ctx->lbuf, 0, need, ctx->stream);
        if (e2 != hipSuccess) {
            (void)hipFree(ctx->lbuf);
            (void)hipFree(ctx->arena);
            delete ctx;
            return fail(nullptr, SF_ERR_HIP, "clearing the learned buffers failed");
        }
    }
    e = hipMemsetAsync(ctx->arena, 0, total, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(ctx->arena);
        delete ctx;
        return fail(nullptr, SF_ERR_HIP, "clearing the arena failed: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return SF_OK;
}

sf_status sf_create(const sf_config* cfg, void* hip_stream, sf_ctx* out) {
    return sf_create_batch(cfg, 1, hip_stream, out);
}

sf_status sf_stream_count(sf_ctx c, int32_t* n) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (!n) return fail(c, SF_ERR_INVALID_ARG, "NULL output");
    *n = c->S;
    return SF_OK;
}

// Lays the levels out again (after a change of cameras, tiles or pass length) and uploads the
// tables.  New device buffers are allocated before the old ones are released, and the context
// takes the new layout only once every allocation has succeeded, so that an allocation
// failure (SF_ERR_OOM) leaves the context as it was.  Set-up work, not per frame.
static sf_status upload_levels(sf_ctx c) {
    Layout nl;
    const size_t need = layout_blocks(c, c->mid, nl);
    float* new_mid = nullptr;
    LevelDev* new_sv = nullptr;
    if (need > c->mid_bytes) {
        hipError_t e = dev_malloc((void**)&new_mid, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, e == hipErrorOutOfMemory ? SF_ERR_OOM : SF_ERR_HIP,
                        "hipMalloc of %zu bytes for split predictions failed", need);
        }
    }
    if (nl.sv.size() > c->sv_cap) {
        hipError_t e = dev_malloc((void**)&new_sv, sizeof(LevelDev) * nl.sv.size());
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (new_mid) (void)hipFree(new_mid);
            return fail(c, e == hipErrorOutOfMemory ? SF_ERR_OOM : SF_ERR_HIP,
                        "hipMalloc of the pass table failed");
        }
    }
    if (new_mid || new_sv) {
        // the old buffers may still be read by enqueued work
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (new_mid) {
            if (c->mid) HIP_TRY(c, hipFree(c->mid));
            c->mid = new_mid;
            c->mid_bytes = need;
        }
        if (new_sv) {
            if (c->sv_dev) HIP_TRY(c, hipFree(c->sv_dev));
            c->sv_dev = new_sv;
            c->sv_cap = nl.sv.size();
        }
        layout_blocks(c, c->mid, nl);   // with the new addresses
    }
    drop_graphs(c);   // captured with the old layout
    c->lv = std::move(nl.lv);
    c->sv = std::move(nl.sv);
    c->step_launches = std::move(nl.launches);
    c->lds_bytes = kLdsBytes;
    HIP_TRY(c, prepare_kernels(c->lds_bytes));
    HIP_TRY(c, hipMemcpyAsync(c->lv_dev, c->lv.data(), sizeof(LevelDev) * c->lv.size(),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->sv_dev, c->sv.data(), sizeof(LevelDev) * c->sv.size(),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SF_OK;
}

// Geometry table of one level of a general grid (Section "Spherical image data structure"):
// level h samples the finest grid eta1 (rows1 x cols1 x 3) at every 2^h-th direction; per
// pixel b1 = P eta_next / |P eta_next| toward the next column (the previous one, negated, in
// the last column), dmu = |P eta_next|, b2 = eta x b1 / |eta x b1| oriented toward the next row
// (away from the previous one in the last row), stored as 9 FP32 planes of rows x gpitch:
// b1/dmu, b2/dmu, eta.  False if two neighbouring directions coincide.
static bool grid_table(const double* eta1, int cols1, int h, int R, int C, int gpitch,
                       std::vector<float>& out) {
    const int sc = 1 << h;
    auto E = [&](int i, int j, double* e) {
        const double* p = eta1 + ((size_t)i * sc * cols1 + (size_t)j * sc) * 3;
        e[0] = p[0];
        e[1] = p[1];
        e[2] = p[2];
    };
    const size_t plane = (size_t)R * gpitch;
    out.assign(9 * plane, 0.0f);
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < C; ++j) {
            double e[3], n[3], q[3], b1[3], b2[3];
            E(i, j, e);
            const bool last_c = j + 1 >= C;
            E(i, last_c ? j - 1 : j + 1, n);
            const double en = e[0] * n[0] + e[1] * n[1] + e[2] * n[2];
            for (int k = 0; k < 3; ++k) q[k] = n[k] - e[k] * en;
            const double dmu = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
            if (!(dmu > 1e-12)) return false;
            for (int k = 0; k < 3; ++k) b1[k] = (last_c ? -q[k] : q[k]) / dmu;
            b2[0] = e[1] * b1[2] - e[2] * b1[1];
            b2[1] = e[2] * b1[0] - e[0] * b1[2];
            b2[2] = e[0] * b1[1] - e[1] * b1[0];
            const double nb = sqrt(b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2]);
            if (!(nb > 1e-12)) return false;
            for (int k = 0; k < 3; ++k) b2[k] /= nb;
            if (R >= 2) {
                const bool last_r = i + 1 >= R;
                double m[3];
                E(last_r ? i - 1 : i + 1, j, m);
                double sgn = b2[0] * m[0] + b2[1] * m[1] + b2[2] * m[2];
                if (last_r) sgn = -sgn;
                if (sgn < 0)
                    for (int k = 0; k < 3; ++k) b2[k] = -b2[k];
            }
            const size_t o = (size_t)i * gpitch + j;
            for (int k = 0; k < 3; ++k) {
                out[k * plane + o] = (float)(b1[k] / dmu);
                out[(3 + k) * plane + o] = (float)(b2[k] / dmu);
                out[(6 + k) * plane + o] = (float)e[k];
            }
        }
    return true;
}

static int grid_pitch(int cols) { return (cols + 63) / 64 * 64; }

// Pinhole rays of a finest level (the closed form of the kernels), for a stream of a batch
// that has no grid of its own when another stream has one.
static void pinhole_rays(const sf_camera* cam, int R, int C, std::vector<double>& eta) {
    eta.resize((size_t)R * C * 3);
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < C; ++j) {
            const double x = (j - cam->cx) / cam->fx, y = (i - cam->cy) / cam->fy;
            const double n = sqrt(x * x + y * y + 1.0);
            double* p = &eta[((size_t)i * C + j) * 3];
            p[0] = x / n;
            p[1] = y / n;
            p[2] = 1.0 / n;
        }
}

sf_status sf_set_cameras(sf_ctx c, const sf_camera* cams) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (!cams) return fail(c, SF_ERR_INVALID_ARG, "NULL camera");
    bool any_grid = false;
    for (int s = 0; s < c->S; ++s) {
        const sf_camera* cam = &cams[s];
        if (!(cam->fx > 0) || !(cam->fy > 0) || !isfinite(cam->fx) || !isfinite(cam->fy) ||
            !isfinite(cam->cx) || !isfinite(cam->cy))
            return fail(c, SF_ERR_INVALID_ARG,
                        "camera %d: fx, fy must be finite and > 0, cx, cy finite", s);
        if (cam->eta) {
            any_grid = true;
            const size_t n = (size_t)c->st[s].cfg.rows * c->st[s].cfg.cols;
            for (size_t p = 0; p < n; ++p) {
                const double* e = cam->eta + 3 * p;
                const double nn = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
                if (!isfinite(nn) || fabs(nn - 1.0) > 1e-6)
                    return fail(c, SF_ERR_INVALID_ARG,
                                "camera %d: eta must hold finite unit vectors (pixel %zu)", s, p);
            }
        }
    }
    // geometry tables of every level of every stream (pinhole streams from their rays) when
    // some stream has a grid; built on the host, allocated before anything is released
    float* new_geo = nullptr;
    std::vector<size_t> geo_off(c->lv.size(), 0);
    if (any_grid) {
        std::vector<float> all, tab;
        std::vector<double> rays;
        for (int s = 0; s < c->S; ++s) {
            const StreamInfo& si = c->st[s];
            const double* eta1 = cams[s].eta;
            if (!eta1) {
                pinhole_rays(&cams[s], si.cfg.rows, si.cfg.cols, rays);
                eta1 = rays.data();
            }
            for (int h = 0; h < si.H; ++h) {
                const LevelDev& L = c->lv[si.e0 + h];
                if (!grid_table(eta1, si.cfg.cols, h, L.rows, L.cols, grid_pitch(L.cols), tab))
                    return fail(c, SF_ERR_INVALID_ARG,
                                "camera %d: neighbouring directions of level %d coincide", s,
                                h + 1);
                geo_off[si.e0 + h] = all.size();
                all.insert(all.end(), tab.begin(), tab.end());
            }
        }
        hipError_t e = dev_malloc((void**)&new_geo, all.size() * sizeof(float));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, e == hipErrorOutOfMemory ? SF_ERR_OOM : SF_ERR_HIP,
                        "hipMalloc of the geometry tables failed");
        }
        e = hipMemcpy(new_geo, all.data(), all.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(new_geo);
            return hip_fail(c, e, "uploading the geometry tables");
        }
    }
    float* old_geo = c->geo;
    const bool old_grid = c->grid;
    const std::vector<LevelDev> old_lv = c->lv;
    const std::vector<StreamInfo> old_st = c->st;
    for (int s = 0; s < c->S; ++s) {
        StreamInfo& si = c->st[s];
        const sf_camera* cam = &cams[s];
        si.cam[0] = cam->fx; si.cam[1] = cam->fy; si.cam[2] = cam->cx; si.cam[3] = cam->cy;
        const sf_config& cf = si.cfg;
        for (int h = 0; h < si.H; ++h) {
            LevelDev& L = c->lv[si.e0 + h];
            const double sc = ldexp(1.0, h);
            const double fx = cam->fx / sc, fy = cam->fy / sc, cx = cam->cx / sc, cy = cam->cy / sc;
            L.ifx = (float)(1.0 / fx);
            L.ify = (float)(1.0 / fy);
            L.cxn = (float)(cx / fx);
            L.cyn = (float)(cy / fy);
            L.fx = (float)fx;
            L.N = level_steps(cf.max_flow_px, h);
            L.pass_n = L.N;
            L.pass_first = L.pass_last = 1;
            L.Ns = cf.smooth_iters[h];
            L.halo = level_halo(L.N, L.Ns);
            const double dmu0 = 1.0 / sqrt(fx * fx + 1.0);
            L.g1 = (float)(cf.alpha[0] / (dmu0 * dmu0));
            L.g2 = (float)(cf.alpha[1] / (dmu0 * dmu0));
            L.g3 = cf.alpha[2];
            L.g4 = cf.alpha[3];
            L.g5 = cf.alpha[4];
            L.qscale = (float)(1.0 / dmu0);   // half storage keeps flow in pixels per frame
            L.geo = new_geo ? new_geo + geo_off[si.e0 + h] : nullptr;
            L.gpitch = grid_pitch(L.cols);
        }
        si.dt_prev = 0.0;
        si.update_ran = false;
    }
    c->grid = new_geo != nullptr;
    c->geo = new_geo;
    bool old_pin[kMaxStreams];
    memcpy(old_pin, c->grid_pinhole, sizeof old_pin);
    for (int s = 0; s < c->S; ++s) c->grid_pinhole[s] = cams[s].eta == nullptr;
    sf_status s2 = upload_levels(c);
    if (s2 != SF_OK) {
        if (!c->hip_failed) {   // nothing was uploaded: the context stays as it was
            c->lv = old_lv;
            c->st = old_st;
            c->geo = old_geo;
            c->grid = old_grid;
            memcpy(c->grid_pinhole, old_pin, sizeof old_pin);
            if (new_geo) (void)hipFree(new_geo);
        }
        return s2;
    }
    if (old_geo) (void)hipFree(old_geo);   // upload_levels synchronised the stream
    c->recon_pending = false;   // the state restarts
    HIP_TRY(c, hipMemsetAsync(c->numeric, 0, sizeof *c->numeric, c->stream));
    c->camera = true;
    c->frames = 0;
    c->parity = 0;
    return SF_OK;
}

sf_status sf_set_camera(sf_ctx c, const sf_camera* cam) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (c->S != 1) return fail(c, SF_ERR_INVALID_ARG, "a batch context takes sf_set_cameras");
    return sf_set_cameras(c, cam);
}

sf_status sf_set_tile(sf_ctx c, int32_t level, int32_t tw, int32_t th) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (level < 1 || level > c->max_levels) return fail(c, SF_ERR_INVALID_ARG, "level out of range");
    const int h = level - 1;
    if (!(tw == 0 && th == 0)) {
        for (int s = 0; s < c->S; ++s) {
            const StreamInfo& si = c->st[s];
            if (h >= si.H) continue;
            const int halo = last_pass_halo(level_steps(si.cfg.max_flow_px, h),
                                            si.cfg.smooth_iters[h], c->pass_steps);
            if (tw < 1 || th < 1 || tw + 2 * halo > kRegion || th + 2 * halo > kRegion)
                return fail(c, SF_ERR_INVALID_ARG, "tile %dx%d with halo %d exceeds %d", tw, th,
                            halo, kRegion);
        }
    }
    st = flush_recon(c);
    if (st != SF_OK) return st;
    const int old_tw = c->user_tw[h], old_th = c->user_th[h];
    c->user_tw[h] = tw;
    c->user_th[h] = th;
    if (c->camera) {
        sf_status s2 = upload_levels(c);
        if (s2 != SF_OK) {
            c->user_tw[h] = old_tw;
            c->user_th[h] = old_th;
            return s2;
        }
    }
    return SF_OK;
}

sf_status sf_set_pass_steps(sf_ctx c, int32_t steps) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (steps < 1 || steps > 64) return fail(c, SF_ERR_INVALID_ARG, "steps must be in [1, 64]");
    for (int s = 0; s < c->S; ++s) {
        const StreamInfo& si = c->st[s];
        for (int h = 0; h < si.H; ++h) {
            const int halo = last_pass_halo(level_steps(si.cfg.max_flow_px, h),
                                            si.cfg.smooth_iters[h], steps);
            if (2 * halo >= kRegion)
                return fail(c, SF_ERR_UNSUPPORTED, "stream %d level %d: halo %d with %d steps per "
                            "pass exceeds the region", s, h + 1, halo, steps);
        }
    }
    st = flush_recon(c);
    if (st != SF_OK) return st;
    const int old = c->pass_steps;
    c->pass_steps = steps;
    if (c->camera) {
        sf_status s2 = upload_levels(c);
        if (s2 != SF_OK) {
            c->pass_steps = old;
            return s2;
        }
    }
    return SF_OK;
}

// -- timing ---------------------------------------------------------------------------------
static hipEvent_t pool_get(sf_ctx c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct TimedLaunch {
    sf_ctx c;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(sf_ctx c_, int k) : c(c_), kind(k) {
        if (c->timing) {
            a = pool_get(c);
            b = pool_get(c);
            if (a) (void)hipEventRecord(a, c->stream);
        }
    }
    void done() {
        if (c->timing && a && b) {
            (void)hipEventRecord(b, c->stream);
            c->marks.push_back({a, b, kind});
        }
    }
};

// Runs the deferred reconstruction launch, if any.  Every entry point that reads or replaces
// the finest levels' flow, or relays the levels out, calls it first.
static sf_status flush_recon(sf_ctx c) {
    if (!c->recon_pending) return SF_OK;
    c->recon_pending = false;
    const int tile = recon_tile(c, 0);
    ElemArgs r = tile_args(c, 0, 1, c->parity, tile);
    TimedLaunch t(c, 2);
    HIP_TRY(c, launch_reconstruct(c->storage, tile, r, c->stream));
    t.done();
    return SF_OK;
}

sf_status sf_set_timing(sf_ctx c, int32_t enable) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    c->timing = enable != 0;
    return SF_OK;
}

sf_status sf_set_graph(sf_ctx c, int32_t enable) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (!enable) drop_graphs(c);
    c->graph_on = enable != 0;
    return SF_OK;
}

sf_status sf_set_input_stream(sf_ctx c, void* hip_stream) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    if (s == c->stream) s = nullptr;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->pyr_stream) HIP_TRY(c, hipStreamSynchronize(c->pyr_stream));
    if (s && !c->pyr_stream) {
        HIP_TRY(c, hipStreamCreateWithFlags(&c->pyr_stream, hipStreamNonBlocking));
        HIP_TRY(c, hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
        HIP_TRY(c, hipEventCreateWithFlags(&c->ev_pyr, hipEventDisableTiming));
        for (int m = 0; m < 2; ++m)
            HIP_TRY(c, hipEventCreateWithFlags(&c->ev_step[m], hipEventDisableTiming));
    }
    c->in_stream = s;
    c->step_rec[0] = c->step_rec[1] = false;
    return SF_OK;
}

sf_status sf_kernel_times(sf_ctx c, double* ms3, int64_t* launches3, int32_t reset) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (!ms3 || !launches3) return fail(c, SF_ERR_INVALID_ARG, "NULL output");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto& m : c->marks) {
        float ms = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&ms, m.a, m.b));
        c->ms[m.kind] += ms;
        c->launches[m.kind] += 1;
        c->pool.push_back(m.a);
        c->pool.push_back(m.b);
    }
    c->marks.clear();
    for (int k = 0; k < 3; ++k) {
        ms3[k] = c->ms[k];
        launches3[k] = c->launches[k];
    }
    if (reset)
        for (int k = 0; k < 3; ++k) { c->ms[k] = 0.0; c->launches[k] = 0; }
    return SF_OK;
}

// -- learned update -------------------------------------------------------------------------
static PackArgs pack_args(float* params, uint16_t* wf, uint16_t* wb, float* bias) {
    PackArgs p{};
    p.params = params;
    static const int ch[5] = {kCnnInputs, 16, 16, 16, 3};
    int off = 0;
    for (int l = 0; l < kCnnLayers; ++l) {
        p.cin[l] = ch[l];
        p.cout[l] = ch[l + 1];
        p.woff[l] = off;
        off += 9 * ch[l] * ch[l + 1];
        p.boff[l] = off;
        off += ch[l + 1];
    }
    p.wf = wf;
    p.wb = wb;
    p.bias = bias;
    return p;
}

// network on the finest level of every stream, then the per-pixel choice, smoothing and store
static sf_status run_learned(sf_ctx c, int q, hipStream_t strm) {
    NetCombineArgs a{};   // the network on the input the level step packed, then the choice
    a.net.segs = c->segs;
    a.net.in = c->lpack;
    a.net.w = c->wf;
    a.net.bias = c->cnn_bias;
    a.lv = c->lv_dev;
    for (int s = 0; s < c->S; ++s) a.ent[s] = c->st[s].e0;
    a.parity = q;
    a.threshold = c->threshold;
    a.fallbacks = c->fallbacks;
    HIP_TRY(c, launch_net_combine(c->storage, a, strm));
    return SF_OK;
}

sf_status sf_set_learned(sf_ctx c, const float* params, size_t n, float threshold) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (!c->learned) return fail(c, SF_ERR_STATE, "the context was not created with the learned update");
    if (!params) return fail(c, SF_ERR_INVALID_ARG, "NULL parameters");
    if (n != (size_t)kCnnParams) return fail(c, SF_ERR_INVALID_ARG, "expected %d parameters", kCnnParams);
    if (isnan(threshold)) return fail(c, SF_ERR_INVALID_ARG, "threshold must not be NaN");
    for (size_t k = 0; k < n; ++k)
        if (!isfinite(params[k])) return fail(c, SF_ERR_INVALID_ARG, "parameters must be finite");
    HIP_TRY(c, hipMemcpyAsync(c->params_dev, params, n * sizeof(float), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, launch_pack_weights(pack_args(c->params_dev, c->wf, c->wb, c->cnn_bias), c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);   // the threshold is an argument of a captured launch
    c->threshold = threshold;
    c->weights = true;
    return SF_OK;
}

sf_status sf_check_state(sf_ctx c, uint64_t* streams) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (!streams) return fail(c, SF_ERR_INVALID_ARG, "NULL output");
    unsigned long long v = 0;
    HIP_TRY(c, hipMemcpyAsync(&v, c->numeric, sizeof v, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *streams = (uint64_t)v;
    if (!v) return SF_OK;
    HIP_TRY(c, hipMemsetAsync(c->numeric, 0, sizeof v, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int first = 0;
    while (!((v >> first) & 1ull)) ++first;
    return fail(c, SF_ERR_NUMERIC,
                "a stored flow value was not finite (streams mask 0x%llx, first %d) since the "
                "last check", v, first);
}

sf_status sf_learned_stats(sf_ctx c, int64_t* fallbacks, int64_t* pixels, int32_t reset) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (!fallbacks || !pixels) return fail(c, SF_ERR_INVALID_ARG, "NULL output");
    if (!c->learned) return fail(c, SF_ERR_STATE, "not a learned context");
    unsigned long long v = 0;
    HIP_TRY(c, hipMemcpyAsync(&v, c->fallbacks, sizeof v, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *fallbacks = (int64_t)v;
    *pixels = c->learned_pixels;
    if (reset) {
        HIP_TRY(c, hipMemsetAsync(c->fallbacks, 0, sizeof v, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        c->learned_pixels = 0;
    }
    return SF_OK;
}

sf_status sf_get_update_inputs(sf_ctx c, int32_t stream, float* out) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (!c->learned) return fail(c, SF_ERR_STATE, "not a learned context");
    if (stream < 0 || stream >= c->S) return fail(c, SF_ERR_INVALID_ARG, "stream out of range");
    if (!is_device_ptr(out)) return fail(c, SF_ERR_INVALID_ARG, "out must be a device pointer");
    if (c->frames < 2 || !c->st[stream].update_ran)
        return fail(c, SF_ERR_STATE, "no update has run since the camera or the state was set");
    st = flush_recon(c);
    if (st != SF_OK) return st;
    ElemArgs a{};
    a.lv = c->lv_dev;
    a.n = 1;
    a.ent[0] = c->st[stream].e0;
    a.blk[0] = 0;
    const LevelDev& L = c->lv[a.ent[0]];
    a.blk[1] = (L.rows * L.cols + kElemBlock - 1) / kElemBlock;
    a.parity = c->parity;
    a.out = out;
    HIP_TRY(c, launch_learned_extract(c->storage, a, c->stream));
    return SF_OK;
}

// -- frames ---------------------------------------------------------------------------------
// The pyramid launches of a frame on stream strm: finest to coarsest, one launch per two depths
// (d, d + 1) for all streams.  With `rec`, the launches that read the frame's inputs are noted
// (for a frame graph's node updates).
static sf_status enqueue_pyramid(sf_ctx c, const FrameInputs& in, hipStream_t strm,
                                 std::vector<sf_ctx_s::FrameArgsNode>* rec) {
    for (int h = 1; h < c->max_levels; h += 2) {
        const int tile = big_tile(c, h, 0);
        ElemArgs a = tile_args(c, h, 0, 0, tile);
        a.in = in;
        if (a.n == 0) continue;
        if (rec) {
            rec->emplace_back();
            rec->back().kind = 1;
            rec->back().e = a;
        }
        TimedLaunch t(c, 0);
        HIP_TRY(c, launch_pyramid(c->storage, tile, a, strm));
        t.done();
    }
    return SF_OK;
}

// Every launch of a frame after the first on stream strm: the pyramid (unless it was enqueued
// on the pyramid stream), the level-step launches
// (reading the state of `parity`), the learned update, and the reconstruction of all but the
// finest pair of levels (that one waits: recon_pending).
static sf_status enqueue_frame(sf_ctx c, const FrameInputs& in, bool inertial,
                               const Inertial* imu, int parity, hipStream_t strm,
                               std::vector<sf_ctx_s::FrameArgsNode>* rec,
                               bool with_pyramid = true) {
    sf_status st = with_pyramid ? enqueue_pyramid(c, in, strm, rec) : SF_OK;
    if (st != SF_OK) return st;
    for (const auto& sl : c->step_launches) {
        StepArgs a{};
        a.lv = c->sv_dev + sl.e0;
        a.nent = sl.n;
        a.parity = parity;
        a.in = in;
        if (inertial) memcpy(a.imu, imu, sizeof a.imu);
        if (rec) {
            rec->emplace_back();
            rec->back().kind = 2;
            rec->back().st = a;
        }
        TimedLaunch t(c, 1);
        HIP_TRY(c, launch_step(c->storage, inertial, c->grid, a, sl.nblocks, c->lds_bytes, strm));
        t.done();
    }
    const int q = 1 - parity;
    if (c->learned) {
        st = run_learned(c, q, strm);
        if (st != SF_OK) return st;
    }
    // reconstruction, coarse to fine: one launch per two levels (h + 1, h), h even, for the
    // streams where h is below the top (the launch holding level 0 is deferred)
    for (int h = (c->max_levels - 2) & ~1; h > 0; h -= 2) {
        const int tile = recon_tile(c, h);
        ElemArgs r = tile_args(c, h, 1, q, tile);
        TimedLaunch t(c, 2);
        HIP_TRY(c, launch_reconstruct(c->storage, tile, r, strm));
        t.done();
    }
    return SF_OK;
}

// Releases the frame graphs (after the work already launched from them has finished).
static void drop_graphs(sf_ctx c) {
    bool any = false;
    for (auto& byp : c->graphs)
        for (auto& fg : byp) any = any || fg.x || fg.g;
    if (!any) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& byp : c->graphs)
        for (auto& fg : byp) {
            if (fg.x) (void)hipGraphExecDestroy(fg.x);
            if (fg.g) (void)hipGraphDestroy(fg.g);
            fg = sf_ctx_s::FrameGraph{};
        }
}

// Captures the frame's launches into the graph for (parity, inertial) on the private stream and
// finds, in launch order, the kernel nodes whose arguments change from frame to frame.
static sf_status capture_frame(sf_ctx c, sf_ctx_s::FrameGraph& fg, const FrameInputs& in,
                               bool inertial, const Inertial* imu) {
    if (!c->cap) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    std::vector<sf_ctx_s::FrameArgsNode> rec;
    HIP_TRY(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    sf_status st = enqueue_frame(c, in, inertial, imu, c->parity, c->cap, &rec);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap, &g);
    if (st != SF_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != SF_OK ? st : hip_fail(c, e, "hipStreamEndCapture");
    }
    // the capture on one stream is a chain: walk it from its root
    std::vector<hipGraphNode_t> order;
    size_t nroot = 0;
    e = hipGraphGetRootNodes(g, nullptr, &nroot);
    if (e == hipSuccess && nroot == 1) {
        hipGraphNode_t n = nullptr;
        e = hipGraphGetRootNodes(g, &n, &nroot);
        while (e == hipSuccess && n) {
            order.push_back(n);
            size_t nd = 0;
            e = hipGraphNodeGetDependentNodes(n, nullptr, &nd);
            if (e != hipSuccess || nd == 0) break;
            if (nd != 1) { e = hipErrorInvalidValue; break; }
            e = hipGraphNodeGetDependentNodes(n, &n, &nd);
        }
    } else if (e == hipSuccess) {
        e = hipErrorInvalidValue;
    }
    size_t k = 0;
    for (size_t i = 0; e == hipSuccess && i < order.size(); ++i) {
        hipGraphNodeType t;
        e = hipGraphNodeGetType(order[i], &t);
        if (e != hipSuccess || t != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams p{};
        e = hipGraphKernelNodeGetParams(order[i], &p);
        if (e != hipSuccess) break;
        const int kind = frame_input_kind(p.func);
        if (kind == 0) continue;
        if (k >= rec.size() || rec[k].kind != kind) { e = hipErrorInvalidValue; break; }
        rec[k].node = order[i];
        rec[k].p = p;
        ++k;
    }
    if (e == hipSuccess && k != rec.size()) e = hipErrorInvalidValue;
    hipGraphExec_t x = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(c, e, "capturing the frame graph");
    }
    fg.g = g;
    fg.x = x;
    fg.nodes = std::move(rec);
    return SF_OK;
}

// A frame after the first through the frame graph of the current parity: captured on first
// use, then its pyramid and level-step nodes take this frame's inputs and it is launched on the
// context stream.
static sf_status replay_frame(sf_ctx c, const FrameInputs& in, bool inertial,
                              const Inertial* imu) {
    sf_ctx_s::FrameGraph& fg = c->graphs[c->parity][inertial ? 1 : 0];
    if (!fg.x) {
        sf_status st = capture_frame(c, fg, in, inertial, imu);
        if (st != SF_OK) return st;
    }
    for (auto& nd : fg.nodes) {
        void* args[1];
        if (nd.kind == 1) {
            nd.e.in = in;
            args[0] = &nd.e;
        } else {
            nd.st.in = in;
            if (inertial) memcpy(nd.st.imu, imu, sizeof nd.st.imu);
            args[0] = &nd.st;
        }
        hipKernelNodeParams p = nd.p;
        p.kernelParams = args;
        p.extra = nullptr;
        HIP_TRY(c, hipGraphExecKernelNodeSetParams(fg.x, nd.node, &p));
    }
    HIP_TRY(c, hipGraphLaunch(fg.x, c->stream));
    return SF_OK;
}

// A frame of every stream; omega, omega_dot and acc (host, 3 values per stream, or NULL for
// zeros) are the camera rates of the inertial source terms, or all NULL for the paper's
// prediction.
static sf_status push_frames(sf_ctx c, const void* const* Y, const void* const* rho,
                             const double* dt, const double* omega, const double* omega_dot,
                             const double* acc) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (!c->camera) return fail(c, SF_ERR_STATE, "the cameras must be set before pushing");
    if (c->learned && !c->weights)
        return fail(c, SF_ERR_STATE, "the learned update needs sf_set_learned before pushing");
    if (!Y || !rho || !dt) return fail(c, SF_ERR_INVALID_ARG, "NULL argument array");
    for (int s = 0; s < c->S; ++s) {
        if (!is_device_ptr(Y[s]) || !is_device_ptr(rho[s]))
            return fail(c, SF_ERR_INVALID_ARG, "stream %d: Y and rho must be device pointers", s);
        if (!(dt[s] > 0.0) || !isfinite(dt[s]))
            return fail(c, SF_ERR_INVALID_ARG, "stream %d: dt must be > 0 and finite", s);
        for (int k = 0; k < 3; ++k)
            if ((omega && !isfinite(omega[3 * s + k])) || (acc && !isfinite(acc[3 * s + k])) ||
                (omega_dot && !isfinite(omega_dot[3 * s + k])))
                return fail(c, SF_ERR_INVALID_ARG,
                            "stream %d: omega, omega_dot and acc must be finite", s);
    }
    st = flush_recon(c);
    if (st != SF_OK) return st;
    FrameInputs in{};
    for (int s = 0; s < c->S; ++s) {
        in.Y[s] = Y[s];
        in.R[s] = rho[s];
        const double dp = c->st[s].dt_prev;
        in.scale[s] = (c->frames == 0 || dt[s] == dp) ? 1.0f : (float)(dt[s] / dp);
    }
    in.mbuf = c->mbuf;
    // inputs on the caller's input stream: the pyramid on the library's pyramid stream (frames
    // after the first, eager launches without timing marks), else everything on the context
    // stream after the input stream's work
    const bool ovl = c->in_stream != nullptr;
    const bool side = ovl && c->frames > 0 && !c->timing && !c->graph_on;
    if (ovl) HIP_TRY(c, hipEventRecord(c->ev_in, c->in_stream));
    if (ovl && !side) HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_in, 0));
    if (side) {
        HIP_TRY(c, hipStreamWaitEvent(c->pyr_stream, c->ev_in, 0));
        if (c->step_rec[c->mbuf])
            HIP_TRY(c, hipStreamWaitEvent(c->pyr_stream, c->ev_step[c->mbuf], 0));
        st = enqueue_pyramid(c, in, c->pyr_stream, nullptr);
        if (st != SF_OK) return st;
        HIP_TRY(c, hipEventRecord(c->ev_pyr, c->pyr_stream));
        HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_pyr, 0));
    }
    if (c->frames == 0) {
        st = enqueue_pyramid(c, in, c->stream, nullptr);
        if (st != SF_OK) return st;
        for (int h = 0; h < c->max_levels; ++h) {
            ElemArgs a = elem_args(c, h, 0);
            a.in = in;
            HIP_TRY(c, launch_init(c->storage, a, c->stream));
        }
        c->parity = 0;
    } else {
        // inertial rates in the filter's time unit: Omega dt (rad/frame), dOmega dt^2
        // (rad/frame^2), a dt^2 (1/frame^2)
        Inertial imu[kMaxStreams] = {};
        const bool inertial = omega || omega_dot || acc;
        for (int s = 0; inertial && s < c->S; ++s) {
            const double d = dt[s];
            auto v = [&](const double* base, int k, double scale) {
                return base ? (float)(base[3 * s + k] * scale) : 0.0f;
            };
            imu[s].ox = v(omega, 0, d);
            imu[s].oy = v(omega, 1, d);
            imu[s].oz = v(omega, 2, d);
            imu[s].dx = v(omega_dot, 0, d * d);
            imu[s].dy = v(omega_dot, 1, d * d);
            imu[s].dz = v(omega_dot, 2, d * d);
            imu[s].ax = v(acc, 0, d * d);
            imu[s].ay = v(acc, 1, d * d);
            imu[s].az = v(acc, 2, d * d);
        }
        if (c->graph_on && !c->timing)
            st = replay_frame(c, in, inertial, imu);
        else
            st = enqueue_frame(c, in, inertial, imu, c->parity, c->stream, nullptr, !side);
        if (st != SF_OK) return st;
        if (c->learned)
            for (int s = 0; s < c->S; ++s) {
                const LevelDev& L = c->lv[c->st[s].e0];
                c->learned_pixels += (int64_t)L.rows * L.cols;
            }
        c->recon_pending = c->max_levels >= 2;
        c->parity = 1 - c->parity;
        for (int s = 0; s < c->S; ++s) c->st[s].update_ran = true;
    }
    if (ovl) {
        // this frame's reads end here; the previous frame's inputs are free once the input
        // stream has waited for its record
        HIP_TRY(c, hipEventRecord(c->ev_step[c->mbuf], c->stream));
        c->step_rec[c->mbuf] = true;
        if (c->step_rec[1 - c->mbuf])
            HIP_TRY(c, hipStreamWaitEvent(c->in_stream, c->ev_step[1 - c->mbuf], 0));
    }
    c->mbuf ^= 1;
    for (int s = 0; s < c->S; ++s) c->st[s].dt_prev = dt[s];
    c->frames += 1;
    return SF_OK;
}

sf_status sf_push_frames(sf_ctx c, const void* const* Y, const void* const* rho, const double* dt) {
    return push_frames(c, Y, rho, dt, nullptr, nullptr, nullptr);
}

sf_status sf_push_frames_ex(sf_ctx c, const void* const* Y, const void* const* rho,
                            const double* dt, const double* omega, const double* omega_dot,
                            const double* acc) {
    return push_frames(c, Y, rho, dt, omega, omega_dot, acc);
}

sf_status sf_push_frame(sf_ctx c, const void* Y, const void* rho, double dt) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (c->S != 1) return fail(c, SF_ERR_INVALID_ARG, "a batch context takes sf_push_frames");
    return push_frames(c, &Y, &rho, &dt, nullptr, nullptr, nullptr);
}

sf_status sf_push_frame_ex(sf_ctx c, const void* Y, const void* rho, double dt,
                           const double* omega, const double* omega_dot, const double* acc) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (c->S != 1) return fail(c, SF_ERR_INVALID_ARG, "a batch context takes sf_push_frames_ex");
    return push_frames(c, &Y, &rho, &dt, omega, omega_dot, acc);
}

// Outputs of the streams s with outs[s] set.  With the finest reconstruction pending (and a
// kind that depends on it) it runs now and writes the outputs of the streams it covers; the
// others (single-level streams) get an output launch.
static sf_status write_outputs(sf_ctx c, int32_t kind, float* const* outs) {
    bool covered[kMaxStreams] = {};
    if (kind != SF_FLOW_RHO && c->recon_pending) {
        c->recon_pending = false;
        const int tile = recon_tile(c, 0);
        ElemArgs r = tile_args(c, 0, 1, c->parity, tile);
        r.kind = kind;
        for (int k = 0; k < r.n; ++k) {
            const int s = c->lv[r.ent[k]].stream;
            r.outs[k] = outs[s];
            r.inv_dts[k] = (float)(1.0 / c->st[s].dt_prev);
            covered[s] = true;
        }
        TimedLaunch t(c, 2);
        HIP_TRY(c, launch_reconstruct(c->storage, tile, r, c->stream));
        t.done();
    }
    ElemArgs a{};
    a.lv = c->lv_dev;
    a.parity = c->parity;
    a.kind = kind;
    int b = 0;
    for (int s = 0; s < c->S; ++s) {
        if (!outs[s] || covered[s]) continue;
        const int e = c->st[s].e0;
        a.ent[a.n] = e;
        a.blk[a.n] = b;
        a.outs[a.n] = outs[s];
        a.inv_dts[a.n] = (float)(1.0 / c->st[s].dt_prev);
        b += (c->lv[e].rows * c->lv[e].cols + kElemBlock - 1) / kElemBlock;
        ++a.n;
    }
    a.blk[a.n] = b;
    if (a.n > 0) HIP_TRY(c, launch_output(c->storage, a, c->stream));
    return SF_OK;
}

static sf_status check_pushed(sf_ctx c) {
    if (!c->camera || c->frames == 0) return fail(c, SF_ERR_STATE, "no frame has been pushed");
    return SF_OK;
}

sf_status sf_get_flow_stream(sf_ctx c, int32_t stream, int32_t kind, void* out) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (stream < 0 || stream >= c->S) return fail(c, SF_ERR_INVALID_ARG, "stream out of range");
    if (kind < SF_FLOW_W_RAD_S || kind > SF_FLOW_W_FRAME)
        return fail(c, SF_ERR_INVALID_ARG, "unknown flow kind %d", kind);
    if (!is_device_ptr(out)) return fail(c, SF_ERR_INVALID_ARG, "out must be a device pointer");
    st = check_pushed(c);
    if (st != SF_OK) return st;
    float* outs[kMaxStreams] = {};
    outs[stream] = (float*)out;
    return write_outputs(c, kind, outs);
}

sf_status sf_get_flows(sf_ctx c, int32_t kind, void* const* outs) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (!outs) return fail(c, SF_ERR_INVALID_ARG, "NULL output array");
    if (kind < SF_FLOW_W_RAD_S || kind > SF_FLOW_W_FRAME)
        return fail(c, SF_ERR_INVALID_ARG, "unknown flow kind %d", kind);
    float* o[kMaxStreams] = {};
    for (int s = 0; s < c->S; ++s) {
        if (!outs[s]) continue;
        if (!is_device_ptr(outs[s]))
            return fail(c, SF_ERR_INVALID_ARG, "stream %d: out must be a device pointer", s);
        o[s] = (float*)outs[s];
    }
    st = check_pushed(c);
    if (st != SF_OK) return st;
    return write_outputs(c, kind, o);
}

sf_status sf_get_flow(sf_ctx c, int32_t kind, void* out) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (c->S != 1) return fail(c, SF_ERR_INVALID_ARG, "a batch context takes sf_get_flow_stream");
    return sf_get_flow_stream(c, 0, kind, out);
}

// -- mapping a camera's frame onto a stream's grid ------------------------------------------
sf_status sf_set_source_camera(sf_ctx c, int32_t stream, const sf_camera* src, int32_t rows,
                               int32_t cols) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (stream < 0 || stream >= c->S) return fail(c, SF_ERR_INVALID_ARG, "stream out of range");
    if (!src) return fail(c, SF_ERR_INVALID_ARG, "NULL camera");
    if (!(src->fx > 0) || !(src->fy > 0) || !isfinite(src->fx) || !isfinite(src->fy) ||
        !isfinite(src->cx) || !isfinite(src->cy))
        return fail(c, SF_ERR_INVALID_ARG, "fx, fy must be finite and > 0, cx, cy finite");
    if (src->eta) return fail(c, SF_ERR_INVALID_ARG, "the source camera is a pinhole (eta NULL)");
    if (rows < 2 || cols < 2 || rows > (1 << 15) || cols > (1 << 15))
        return fail(c, SF_ERR_INVALID_ARG, "source size must be in [2, 32768]");
    StreamInfo& si = c->st[stream];
    si.source = true;
    si.src[0] = src->fx;
    si.src[1] = src->fy;
    si.src[2] = src->cx;
    si.src[3] = src->cy;
    si.src_rows = rows;
    si.src_cols = cols;
    return SF_OK;
}

sf_status sf_map_frame(sf_ctx c, int32_t stream, const void* Y_src, const void* rho_src,
                       void* Y_out, void* rho_out) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (stream < 0 || stream >= c->S) return fail(c, SF_ERR_INVALID_ARG, "stream out of range");
    const StreamInfo& si = c->st[stream];
    if (!c->camera) return fail(c, SF_ERR_STATE, "the cameras must be set before mapping");
    if (!si.source) return fail(c, SF_ERR_STATE, "no source camera set for stream %d", stream);
    if (!is_device_ptr(Y_src) || !is_device_ptr(rho_src) || !is_device_ptr(Y_out) ||
        !is_device_ptr(rho_out))
        return fail(c, SF_ERR_INVALID_ARG, "images must be device pointers");
    MapArgs a{};
    a.lv = c->lv_dev;
    a.ent = si.e0;
    a.fx = (float)si.src[0];
    a.fy = (float)si.src[1];
    a.cx = (float)si.src[2];
    a.cy = (float)si.src[3];
    a.rows = si.src_rows;
    a.cols = si.src_cols;
    a.Y = Y_src;
    a.R = rho_src;
    a.Yout = Y_out;
    a.Rout = rho_out;
    HIP_TRY(c, launch_map(c->storage, a, si.cfg.rows * si.cfg.cols, c->stream));
    return SF_OK;
}

// -- inverse depth from a stereo pair ----------------------------------------------------------
sf_status sf_set_stereo(sf_ctx c, int32_t stream, double baseline, int32_t max_disparity,
                        int32_t iterations, double texture, double residual) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (stream < 0 || stream >= c->S) return fail(c, SF_ERR_INVALID_ARG, "stream out of range");
    if (!(baseline > 0.0) || !isfinite(baseline))
        return fail(c, SF_ERR_INVALID_ARG, "baseline must be finite and > 0");
    if (max_disparity < 0 || max_disparity > 64)
        return fail(c, SF_ERR_INVALID_ARG, "max_disparity must be in [0, 64]");
    if (iterations < 0 || iterations > 16)
        return fail(c, SF_ERR_INVALID_ARG, "iterations must be in [0, 16]");
    if (!(texture >= 0.0) || !isfinite(texture) || !(residual > 0.0) || !isfinite(residual))
        return fail(c, SF_ERR_INVALID_ARG, "texture must be >= 0 and residual > 0, both finite");
    StreamInfo& si = c->st[stream];
    si.stereo = true;
    si.baseline = baseline;
    si.dmax = max_disparity;
    si.iters = iterations;
    si.texture = texture;
    si.residual = residual;
    return SF_OK;
}

sf_status sf_stereo_depth(sf_ctx c, int32_t stream, const void* Y_left, const void* Y_right,
                          void* rho_out) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (stream < 0 || stream >= c->S) return fail(c, SF_ERR_INVALID_ARG, "stream out of range");
    if (!c->camera) return fail(c, SF_ERR_STATE, "the cameras must be set first");
    const StreamInfo& si = c->st[stream];
    if (!si.stereo) return fail(c, SF_ERR_STATE, "no stereo parameters set for stream %d", stream);
    if (c->lv[si.e0].geo && !c->grid_pinhole[stream])
        return fail(c, SF_ERR_UNSUPPORTED, "stereo depth needs a pinhole stream (no eta grid)");
    if (!is_device_ptr(Y_left) || !is_device_ptr(Y_right) || !is_device_ptr(rho_out))
        return fail(c, SF_ERR_INVALID_ARG, "images must be device pointers");
    StereoArgs a{};
    a.YL = Y_left;
    a.YR = Y_right;
    a.rho = rho_out;
    a.rows = si.cfg.rows;
    a.cols = si.cfg.cols;
    a.fx = (float)si.cam[0];
    a.fy = (float)si.cam[1];
    a.cx = (float)si.cam[2];
    a.cy = (float)si.cam[3];
    a.baseline = (float)si.baseline;
    a.dmax = si.dmax;
    a.iters = si.iters;
    a.texture = (float)si.texture;
    a.residual = (float)si.residual;
    HIP_TRY(c, launch_stereo(c->storage, a, c->stream));
    return SF_OK;
}

// -- state blob -----------------------------------------------------------------------------
struct BlobHeader {
    uint32_t magic;
    uint32_t version;
    int32_t levels;
    int32_t initialised;
    double dt_prev;
    int64_t frames;
};
static_assert(sizeof(BlobHeader) == 32, "blob header is 32 bytes");
static_assert(kLearnInputs == kCnnInputs, "the step kernel writes the network's inputs");
static const uint32_t kMagic = 0x54535346u;   // 'SFST'

static size_t blob_bytes(sf_ctx c, int s) {
    size_t n = sizeof(BlobHeader);
    const StreamInfo& si = c->st[s];
    for (int h = 0; h < si.H; ++h) {
        const LevelDev& L = c->lv[si.e0 + h];
        n += (size_t)(L.top ? 5 : 8) * L.rows * L.cols * sizeof(float);
    }
    return n;
}

static float half_to_float(uint16_t h) {
    const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
    uint32_t exp = (h >> 10) & 0x1fu;
    uint32_t man = h & 0x3ffu;
    uint32_t bits;
    if (exp == 0) {
        if (man == 0) {
            bits = sign;
        } else {   // subnormal: renormalise
            int e = -1;
            do { ++e; man <<= 1; } while (!(man & 0x400u));
            bits = sign | ((uint32_t)(127 - 15 - e) << 23) | ((man & 0x3ffu) << 13);
        }
    } else if (exp == 31) {
        bits = sign | 0x7f800000u | (man << 13);
    } else {
        bits = sign | ((exp + 127 - 15) << 23) | (man << 13);
    }
    float f;
    memcpy(&f, &bits, 4);
    return f;
}

static uint16_t float_to_half(float f) {   // round to nearest even
    uint32_t x;
    memcpy(&x, &f, 4);
    const uint32_t sign = (x >> 16) & 0x8000u;
    const uint32_t ax = x & 0x7fffffffu;
    if (ax >= 0x7f800000u) return (uint16_t)(sign | 0x7c00u | (ax > 0x7f800000u ? 0x200u : 0));
    if (ax >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);          // overflow -> inf
    if (ax < 0x38800000u) {                                              // subnormal or zero
        if (ax < 0x33000000u) return (uint16_t)sign;
        const uint32_t e = ax >> 23;
        const uint32_t m = (ax & 0x7fffffu) | 0x800000u;
        const uint32_t shift = 126 - e;                                  // 14..24
        const uint32_t rem = m & ((1u << shift) - 1);
        const uint32_t half = 1u << (shift - 1);
        uint32_t q = m >> shift;
        if (rem > half || (rem == half && (q & 1))) ++q;
        return (uint16_t)(sign | q);
    }
    uint32_t q = ((ax - 0x38000000u) >> 13);
    const uint32_t rem = ax & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (q & 1))) ++q;
    return (uint16_t)(sign | q);
}

static sf_status copy_plane(sf_ctx c, bool to_host, void* dev, int pitch, int rows, int cols,
                            float* host, float mul, std::vector<uint16_t>& scratch) {
    if (c->esize == 4) {
        if (to_host) {
            HIP_TRY(c, hipMemcpy2DAsync(host, cols * 4, dev, (size_t)pitch * 4, cols * 4, rows,
                                        hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            if (mul != 1.0f)
                for (size_t k = 0; k < (size_t)rows * cols; ++k) host[k] *= mul;
        } else {
            std::vector<float> tmp(host, host + (size_t)rows * cols);
            if (mul != 1.0f)
                for (auto& v : tmp) v *= mul;
            HIP_TRY(c, hipMemcpy2DAsync(dev, (size_t)pitch * 4, tmp.data(), cols * 4, cols * 4,
                                        rows, hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
        }
        return SF_OK;
    }
    scratch.resize((size_t)rows * cols);
    if (to_host) {
        HIP_TRY(c, hipMemcpy2DAsync(scratch.data(), cols * 2, dev, (size_t)pitch * 2, cols * 2,
                                    rows, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (size_t k = 0; k < scratch.size(); ++k) host[k] = half_to_float(scratch[k]) * mul;
    } else {
        for (size_t k = 0; k < scratch.size(); ++k) scratch[k] = float_to_half(host[k] * mul);
        HIP_TRY(c, hipMemcpy2DAsync(dev, (size_t)pitch * 2, scratch.data(), cols * 2, cols * 2,
                                    rows, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return SF_OK;
}

static sf_status transfer_state(sf_ctx c, int s, bool to_host, float* f) {
    std::vector<uint16_t> scratch;
    const StreamInfo& si = c->st[s];
    for (int h = 0; h < si.H; ++h) {
        LevelDev& L = c->lv[si.e0 + h];
        const size_t n = (size_t)L.rows * L.cols;
        const float fin = c->esize == 2 ? 1.0f / L.qscale : 1.0f;    // stored -> rad/frame
        const float mul = to_host ? fin : 1.0f / fin;
        const int par = c->parity;
        for (int k = 0; k < 3; ++k, f += n) {
            sf_status s = copy_plane(c, to_host, L.w[par][k], L.pitch, L.rows, L.cols, f, mul, scratch);
            if (s != SF_OK) return s;
        }
        if (!L.top)
            for (int k = 0; k < 3; ++k, f += n) {
                sf_status s = copy_plane(c, to_host, L.dw[par][k], L.pitch, L.rows, L.cols, f, mul,
                                         scratch);
                if (s != SF_OK) return s;
            }
        sf_status s = copy_plane(c, to_host, L.rho[par], L.pitch, L.rows, L.cols, f, 1.0f, scratch);
        if (s != SF_OK) return s;
        f += n;
        s = copy_plane(c, to_host, L.Y[par], L.pitch, L.rows, L.cols, f, 1.0f, scratch);
        if (s != SF_OK) return s;
        f += n;
    }
    return SF_OK;
}

sf_status sf_state_size_stream(sf_ctx c, int32_t stream, size_t* bytes) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (!bytes) return fail(c, SF_ERR_INVALID_ARG, "NULL output");
    if (stream < 0 || stream >= c->S) return fail(c, SF_ERR_INVALID_ARG, "stream out of range");
    *bytes = blob_bytes(c, stream);
    return SF_OK;
}

sf_status sf_get_state_stream(sf_ctx c, int32_t stream, void* host_blob, size_t bytes) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (stream < 0 || stream >= c->S) return fail(c, SF_ERR_INVALID_ARG, "stream out of range");
    if (!host_blob) return fail(c, SF_ERR_INVALID_ARG, "NULL blob");
    if (bytes != blob_bytes(c, stream))
        return fail(c, SF_ERR_INVALID_ARG, "blob must be %zu bytes", blob_bytes(c, stream));
    if (!c->camera) return fail(c, SF_ERR_STATE, "no camera set");
    const StreamInfo& si = c->st[stream];
    BlobHeader hd{kMagic, 1u, si.H, c->frames > 0 ? 1 : 0, si.dt_prev, c->frames};
    memcpy(host_blob, &hd, sizeof hd);
    if (c->frames == 0) {
        memset((char*)host_blob + sizeof hd, 0, bytes - sizeof hd);
        return SF_OK;
    }
    st = flush_recon(c);
    if (st != SF_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return transfer_state(c, stream, true, (float*)((char*)host_blob + sizeof hd));
}

sf_status sf_set_state_stream(sf_ctx c, int32_t stream, const void* host_blob, size_t bytes) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (stream < 0 || stream >= c->S) return fail(c, SF_ERR_INVALID_ARG, "stream out of range");
    if (!host_blob) return fail(c, SF_ERR_INVALID_ARG, "NULL blob");
    if (bytes != blob_bytes(c, stream))
        return fail(c, SF_ERR_INVALID_ARG, "blob must be %zu bytes", blob_bytes(c, stream));
    if (!c->camera) return fail(c, SF_ERR_STATE, "no camera set");
    BlobHeader hd;
    memcpy(&hd, host_blob, sizeof hd);
    StreamInfo& si = c->st[stream];
    if (hd.magic != kMagic || hd.version != 1u || hd.levels != si.H)
        return fail(c, SF_ERR_INVALID_ARG, "blob header does not match this stream");
    if (hd.initialised && !(hd.dt_prev > 0.0 && isfinite(hd.dt_prev)))
        return fail(c, SF_ERR_INVALID_ARG, "blob dt_prev must be > 0");
    if (c->S > 1 && (!hd.initialised || c->frames == 0))
        return fail(c, SF_ERR_STATE, "a batch takes states only once every stream has a frame");
    st = flush_recon(c);   // the other streams' finest levels
    if (st != SF_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (!hd.initialised) {
        c->recon_pending = false;
        c->frames = 0;
        c->parity = 0;
        return SF_OK;
    }
    std::vector<float> tmp((bytes - sizeof hd) / sizeof(float));
    memcpy(tmp.data(), (const char*)host_blob + sizeof hd, bytes - sizeof hd);
    sf_status s2 = transfer_state(c, stream, false, tmp.data());
    if (s2 != SF_OK) return s2;
    si.update_ran = false;
    if (c->learned) {
        // the learned correction of the output belongs to the frame before the new state:
        // clear it, as the first frame does, so that the flow read back is the state's
        const LevelDev& L = c->lv[si.e0];
        const size_t P = (size_t)c->segs.total;
        for (int k = 0; k < 3; ++k)
            HIP_TRY(c, hipMemsetAsync(c->lbuf + (size_t)(kLearnCorr + k) * P + L.lbase, 0,
                                      (size_t)L.rows * L.cols * sizeof(float), c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    if (c->S == 1) c->frames = std::max<int64_t>(1, hd.frames);
    si.dt_prev = hd.dt_prev;
    return SF_OK;
}

sf_status sf_state_size(sf_ctx c, size_t* bytes) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (c->S != 1) return fail(c, SF_ERR_INVALID_ARG, "a batch context takes sf_state_size_stream");
    return sf_state_size_stream(c, 0, bytes);
}

sf_status sf_get_state(sf_ctx c, void* host_blob, size_t bytes) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (c->S != 1) return fail(c, SF_ERR_INVALID_ARG, "a batch context takes sf_get_state_stream");
    return sf_get_state_stream(c, 0, host_blob, bytes);
}

sf_status sf_set_state(sf_ctx c, const void* host_blob, size_t bytes) {
    sf_status st = check_alive(c);
    if (st != SF_OK) return st;
    if (c->S != 1) return fail(c, SF_ERR_INVALID_ARG, "a batch context takes sf_set_state_stream");
    return sf_set_state_stream(c, 0, host_blob, bytes);
}

sf_status sf_destroy(sf_ctx c) {
    if (!c) return SF_OK;
    (void)hipStreamSynchronize(c->stream);
    if (c->pyr_stream) (void)hipStreamSynchronize(c->pyr_stream);
    for (auto& m : c->marks) { (void)hipEventDestroy(m.a); (void)hipEventDestroy(m.b); }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    if (c->arena) (void)hipFree(c->arena);
    if (c->lbuf) (void)hipFree(c->lbuf);
    if (c->mid) (void)hipFree(c->mid);
    if (c->sv_dev) (void)hipFree(c->sv_dev);
    if (c->geo) (void)hipFree(c->geo);
    drop_graphs(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->pyr_stream) (void)hipStreamDestroy(c->pyr_stream);
    for (hipEvent_t e : {c->ev_in, c->ev_pyr, c->ev_step[0], c->ev_step[1]})
        if (e) (void)hipEventDestroy(e);
    delete c;
    return SF_OK;
}

const char* sf_last_error(sf_ctx c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

}  // extern "C"
