// Host side of the learned update's trainer (sf_net_* in include/sflow.h): the network over a
// list of images, forward pass, Charbonnier endpoint loss, backward pass and Adam, all in the
// kernels of sflow_cnn.hip on the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>

#include "sflow_cnn.h"
#include "sflow_internal.h"

using namespace sflow;

struct sf_net_s {
    hipStream_t stream = nullptr;
    CnnSegs segs{};
    int64_t pixels = 0;             // unpadded pixels over all images
    bool hip_failed = false;
    std::string err;
    char* mem = nullptr;
    float* params = nullptr;        // FP32 master [kCnnParams]
    float* m = nullptr;             // Adam moments
    float* v = nullptr;
    float* grad = nullptr;
    float* dw = nullptr;            // [4][9][16][16]
    float* db = nullptr;            // [4][16]
    uint16_t* wf = nullptr;         // BF16 [4][9][16][16]
    uint16_t* wb = nullptr;
    float* bias = nullptr;          // [4][16]
    float* in = nullptr;            // [kCnnInputs][total]
    float* tgt = nullptr;           // [3][total]
    float* out = nullptr;           // [3][total]
    uint16_t* act[4] = {};          // layer inputs, BF16 NHWC 16
    uint16_t* g[2] = {};            // input gradients
    uint16_t* dout = nullptr;
    float* loss = nullptr;
    int64_t step = 0;
    bool has_params = false;
    float eps = 1e-3f;              // Charbonnier epsilon of the loss, pixels
};

// text of the last failure of a call without a network (sf_net_create,
// sf_net_forward_noalloc); a fixed buffer, so that reporting an error allocates nothing
static char g_net_create_error[512];

static sf_status nfail(sf_net n, sf_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (n) n->err = buf; else memcpy(g_net_create_error, buf, sizeof buf);
    return s;
}

#define NET_TRY(net, expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            (net)->hip_failed = true;                                                   \
            return nfail((net), SF_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));    \
        }                                                                               \
    } while (0)

static bool dev_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

static sf_status net_alive(sf_net n) {
    if (!n) return nfail(nullptr, SF_ERR_INVALID_ARG, "NULL network");
    if (n->hip_failed) return nfail(n, SF_ERR_HIP, "network unusable after a HIP failure: %s",
                                    n->err.c_str());
    return SF_OK;
}

static void layer_offsets(int woff[4], int boff[4], int cin[4], int cout[4]) {
    static const int ch[5] = {kCnnInputs, 16, 16, 16, 3};
    int off = 0;
    for (int l = 0; l < kCnnLayers; ++l) {
        cin[l] = ch[l];
        cout[l] = ch[l + 1];
        woff[l] = off;
        off += 9 * ch[l] * ch[l + 1];
        boff[l] = off;
        off += ch[l + 1];
    }
}

static hipError_t repack(sf_net n) {
    PackArgs p{};
    layer_offsets(p.woff, p.boff, p.cin, p.cout);
    p.params = n->params;
    p.wf = n->wf;
    p.wb = n->wb;
    p.bias = n->bias;
    return launch_pack_weights(p, n->stream);
}

// forward pass over the images already in n->in; leaves the layer inputs in act[] and the
// output planes in n->out
static sf_status forward(sf_net n) {
    const int P = n->segs.total;
    NET_TRY(n, launch_pack_inputs(n->in, kCnnInputs, P, n->act[0], n->stream));
    for (int l = 0; l < kCnnLayers; ++l) {
        ConvArgs a{};
        a.segs = n->segs;
        a.in = n->act[l];
        a.w = n->wf + (size_t)l * 9 * 256;
        a.bias = n->bias + l * 16;
        a.relu = l < kCnnLayers - 1;
        a.nout = l < kCnnLayers - 1 ? 16 : 3;
        a.out = l < kCnnLayers - 1 ? n->act[l + 1] : nullptr;
        a.out_f32 = n->out;
        NET_TRY(n, launch_conv(a, l == kCnnLayers - 1, n->stream));
    }
    return SF_OK;
}

// ---- the forward pass without allocation (sf_net_forward_noalloc) ---------------------------
// Its buffers live in one file-scope device array, `scratch`, laid out for one image of at
// most SF_NOALLOC_MAX_PIXELS pixels: the packed weights (forward and input-gradient BF16
// [4][9][16][16], the latter unused but written by the packing kernel), the biases, the input
// planes, two ping-pong BF16 NHWC activation buffers and the output planes.  Every call
// rewrites every byte it reads (the input planes' padding included), so nothing needs
// clearing between calls.  Host code never passes `scratch` itself to a kernel: its name is a
// host-side stand-in; the device address comes from hipGetSymbolAddress, taken once per device.
namespace {
constexpr size_t al256(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t kNaPx = SF_NOALLOC_MAX_PIXELS;    // a multiple of 16
static_assert(kNaPx % 16 == 0, "the padded image must fit");
constexpr size_t kNaWf = 0;
constexpr size_t kNaWb = kNaWf + al256(4 * 9 * 256 * sizeof(uint16_t));
constexpr size_t kNaBias = kNaWb + al256(4 * 9 * 256 * sizeof(uint16_t));
constexpr size_t kNaIn = kNaBias + al256(4 * 16 * sizeof(float));
constexpr size_t kNaAct0 = kNaIn + al256((size_t)kCnnInputs * kNaPx * sizeof(float));
constexpr size_t kNaAct1 = kNaAct0 + al256(kNaPx * 16 * sizeof(uint16_t));
constexpr size_t kNaOut = kNaAct1 + al256(kNaPx * 16 * sizeof(uint16_t));
constexpr size_t kNaBytes = kNaOut + al256(3 * kNaPx * sizeof(float));
constexpr int kNaMaxDevices = 64;

__device__ __align__(256) char scratch[kNaBytes];

std::mutex g_na_mu;
char* g_na_ptr[kNaMaxDevices] = {};   // device address of `scratch` per device

// the current device's address of `scratch` (looked up on the first call on that device)
hipError_t noalloc_scratch(char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_na_ptr[dev] = (char*)p;
    }
    *out = g_na_ptr[dev];
    return hipSuccess;
}
}  // namespace

extern "C" {

sf_status sf_net_create(const int32_t* rows, const int32_t* cols, int32_t n_images,
                        void* hip_stream, sf_net* out) {
    if (!out) return nfail(nullptr, SF_ERR_INVALID_ARG, "NULL output pointer");
    *out = nullptr;
    if (!rows || !cols) return nfail(nullptr, SF_ERR_INVALID_ARG, "NULL size arrays");
    if (n_images < 1 || n_images > kCnnMaxSegs)
        return nfail(nullptr, SF_ERR_INVALID_ARG, "image count must be in [1, %d]", kCnnMaxSegs);
    sf_net n = new (std::nothrow) sf_net_s;
    if (!n) return nfail(nullptr, SF_ERR_OOM, "host allocation failed");
    n->stream = (hipStream_t)hip_stream;
    CnnSegs& sg = n->segs;
    sg.n = n_images;
    int64_t b = 0, o = 0;
    for (int k = 0; k < n_images; ++k) {
        if (rows[k] < 1 || cols[k] < 1 || (int64_t)rows[k] * cols[k] > (1 << 26)) {
            delete n;
            return nfail(nullptr, SF_ERR_INVALID_ARG, "image %d: size must be in [1, 2^26] pixels", k);
        }
        sg.base[k] = (int)b;
        sg.off[k] = (int)o;
        sg.rows[k] = rows[k];
        sg.cols[k] = cols[k];
        const int64_t npx = (int64_t)rows[k] * cols[k];
        b += (npx + 15) / 16 * 16;
        o += npx;
        if (b > (1 << 27)) {
            delete n;
            return nfail(nullptr, SF_ERR_INVALID_ARG, "at most 2^27 pixels per network batch");
        }
    }
    sg.base[n_images] = (int)b;
    sg.off[n_images] = (int)o;
    sg.total = (int)b;
    n->pixels = o;

    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t P = (size_t)b;
    const size_t sizes[] = {
        kCnnParams * 4, kCnnParams * 4, kCnnParams * 4, kCnnParams * 4,   // params m v grad
        4 * 9 * 256 * 4, 4 * 16 * 4,                                      // dw db
        4 * 9 * 256 * 2, 4 * 9 * 256 * 2, 4 * 16 * 4,                     // wf wb bias
        kCnnInputs * P * 4, 3 * P * 4, 3 * P * 4,                         // in tgt out
        P * 32, P * 32, P * 32, P * 32, P * 32, P * 32, P * 32,           // act[4] g[2] dout
        256};                                                             // loss
    size_t total = 0;
    for (size_t s : sizes) total += al(s);
    hipError_t e = dev_malloc((void**)&n->mem, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete n;
        return nfail(nullptr, e == hipErrorOutOfMemory ? SF_ERR_OOM : SF_ERR_HIP,
                     "hipMalloc of %zu bytes failed: %s", total, hipGetErrorString(e));
    }
    char* q = n->mem;
    int k = 0;
    auto take = [&]() { char* r = q; q += al(sizes[k++]); return r; };
    n->params = (float*)take();
    n->m = (float*)take();
    n->v = (float*)take();
    n->grad = (float*)take();
    n->dw = (float*)take();
    n->db = (float*)take();
    n->wf = (uint16_t*)take();
    n->wb = (uint16_t*)take();
    n->bias = (float*)take();
    n->in = (float*)take();
    n->tgt = (float*)take();
    n->out = (float*)take();
    for (int l = 0; l < 4; ++l) n->act[l] = (uint16_t*)take();
    n->g[0] = (uint16_t*)take();
    n->g[1] = (uint16_t*)take();
    n->dout = (uint16_t*)take();
    n->loss = (float*)take();
    e = hipMemsetAsync(n->mem, 0, total, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) {
        (void)hipFree(n->mem);
        delete n;
        return nfail(nullptr, SF_ERR_HIP, "clearing the network buffers failed: %s",
                     hipGetErrorString(e));
    }
    *out = n;
    return SF_OK;
}

sf_status sf_net_set_params(sf_net n, const float* params, size_t count) {
    sf_status st = net_alive(n);
    if (st != SF_OK) return st;
    if (!params) return nfail(n, SF_ERR_INVALID_ARG, "NULL parameters");
    if (count != (size_t)kCnnParams) return nfail(n, SF_ERR_INVALID_ARG, "expected %d parameters", kCnnParams);
    for (size_t i = 0; i < count; ++i)
        if (!isfinite(params[i])) return nfail(n, SF_ERR_INVALID_ARG, "parameters must be finite");
    NET_TRY(n, hipMemcpyAsync(n->params, params, count * 4, hipMemcpyHostToDevice, n->stream));
    NET_TRY(n, hipMemsetAsync(n->m, 0, kCnnParams * 4, n->stream));
    NET_TRY(n, hipMemsetAsync(n->v, 0, kCnnParams * 4, n->stream));
    NET_TRY(n, repack(n));
    NET_TRY(n, hipStreamSynchronize(n->stream));
    n->step = 0;
    n->has_params = true;
    return SF_OK;
}

sf_status sf_net_get_params(sf_net n, float* params, size_t count) {
    sf_status st = net_alive(n);
    if (st != SF_OK) return st;
    if (!params) return nfail(n, SF_ERR_INVALID_ARG, "NULL output");
    if (count != (size_t)kCnnParams) return nfail(n, SF_ERR_INVALID_ARG, "expected %d parameters", kCnnParams);
    if (!n->has_params) return nfail(n, SF_ERR_STATE, "no parameters set");
    NET_TRY(n, hipMemcpyAsync(params, n->params, count * 4, hipMemcpyDeviceToHost, n->stream));
    NET_TRY(n, hipStreamSynchronize(n->stream));
    return SF_OK;
}

sf_status sf_net_forward(sf_net n, const float* in, float* out) {
    sf_status st = net_alive(n);
    if (st != SF_OK) return st;
    if (!n->has_params) return nfail(n, SF_ERR_STATE, "no parameters set");
    if (!dev_ptr(in) || !dev_ptr(out)) return nfail(n, SF_ERR_INVALID_ARG, "in and out must be device pointers");
    NET_TRY(n, launch_planes_in(n->segs, in, kCnnInputs, n->in, n->stream));
    // inference: the four layers in one launch (bitwise the layer-by-layer pass of training)
    NET_TRY(n, launch_pack_inputs(n->in, kCnnInputs, n->segs.total, n->act[0], n->stream));
    NetArgs a{};
    a.segs = n->segs;
    a.in = n->act[0];
    a.w = n->wf;
    a.bias = n->bias;
    a.out_f32 = n->out;
    NET_TRY(n, launch_net(a, n->stream));
    NET_TRY(n, launch_planes_out(n->segs, n->out, 3, out, n->stream));
    return SF_OK;
}

sf_status sf_net_train_step(sf_net n, const float* in, const float* target, float lr,
                            float* loss_out, float* grad_out) {
    sf_status st = net_alive(n);
    if (st != SF_OK) return st;
    if (!n->has_params) return nfail(n, SF_ERR_STATE, "no parameters set");
    if (!dev_ptr(in) || !dev_ptr(target))
        return nfail(n, SF_ERR_INVALID_ARG, "in and target must be device pointers");
    if (!(lr >= 0.0f) || !isfinite(lr)) return nfail(n, SF_ERR_INVALID_ARG, "lr must be finite and >= 0");
    NET_TRY(n, launch_planes_in(n->segs, in, kCnnInputs, n->in, n->stream));
    NET_TRY(n, launch_planes_in(n->segs, target, 3, n->tgt, n->stream));
    st = forward(n);
    if (st != SF_OK) return st;
    NET_TRY(n, hipMemsetAsync(n->loss, 0, 4, n->stream));
    NET_TRY(n, hipMemsetAsync(n->dw, 0, 4 * 9 * 256 * 4, n->stream));
    NET_TRY(n, hipMemsetAsync(n->db, 0, 4 * 16 * 4, n->stream));
    LossArgs la{};
    la.segs = n->segs;
    la.out = n->out;
    la.target = n->tgt;
    la.eps = n->eps;
    la.inv_count = (float)(1.0 / (double)n->pixels);
    la.loss = n->loss;
    la.dout = n->dout;
    NET_TRY(n, launch_loss(la, n->stream));
    // about 512 waves share the weight-gradient reduction
    const int groups = n->segs.total / 16;
    const int per_wave = groups / 512 + 1;
    const uint16_t* grad_in = n->dout;    // d loss / d output of the current layer
    for (int l = kCnnLayers - 1; l >= 0; --l) {
        DwArgs d{};
        d.segs = n->segs;
        d.in = n->act[l];
        d.dout = grad_in;
        d.act = l < kCnnLayers - 1 ? n->act[l + 1] : nullptr;
        d.per_wave = per_wave;
        d.dw = n->dw + (size_t)l * 9 * 256;
        d.db = n->db + l * 16;
        NET_TRY(n, launch_conv_dw(d, n->stream));
        if (l == 0) break;
        ConvArgs c{};
        c.segs = n->segs;
        c.in = grad_in;
        c.mask = l < kCnnLayers - 1 ? n->act[l + 1] : nullptr;
        c.w = n->wb + (size_t)l * 9 * 256;
        c.relu = 0;
        c.nout = 16;
        uint16_t* dst = n->g[l & 1];
        c.out = dst;
        NET_TRY(n, launch_conv(c, false, n->stream));
        grad_in = dst;
    }
    GradArgs ga{};
    layer_offsets(ga.woff, ga.boff, ga.cin, ga.cout);
    ga.dw = n->dw;
    ga.db = n->db;
    ga.grad = n->grad;
    NET_TRY(n, launch_gather_grads(ga, n->stream));
    if (lr > 0.0f) {
        ++n->step;
        AdamArgs aa{};
        aa.params = n->params;
        aa.grad = n->grad;
        aa.m = n->m;
        aa.v = n->v;
        aa.nparams = kCnnParams;
        aa.lr = lr;
        aa.b1 = 0.9f;
        aa.b2 = 0.999f;
        aa.eps = 1e-8f;
        aa.c1 = (float)(1.0 / (1.0 - pow(0.9, (double)n->step)));
        aa.c2 = (float)(1.0 / (1.0 - pow(0.999, (double)n->step)));
        NET_TRY(n, launch_adam(aa, n->stream));
        NET_TRY(n, repack(n));
    }
    if (loss_out)
        NET_TRY(n, hipMemcpyAsync(loss_out, n->loss, 4, hipMemcpyDeviceToHost, n->stream));
    if (grad_out)
        NET_TRY(n, hipMemcpyAsync(grad_out, n->grad, kCnnParams * 4, hipMemcpyDeviceToHost, n->stream));
    NET_TRY(n, hipStreamSynchronize(n->stream));
    return SF_OK;
}

sf_status sf_net_forward_noalloc(const float* params, int32_t rows, int32_t cols,
                                 const float* in, float* out, void* hip_stream) {
    if (rows < 1 || cols < 1 || (int64_t)rows * cols > (int64_t)kNaPx)
        return nfail(nullptr, SF_ERR_INVALID_ARG,
                     "image size must be in [1, %d] pixels (rows %d, cols %d)",
                     (int)kNaPx, rows, cols);
    if (!dev_ptr(params) || !dev_ptr(in) || !dev_ptr(out))
        return nfail(nullptr, SF_ERR_INVALID_ARG, "params, in and out must be device pointers");
    char* base = nullptr;
    hipError_t e = noalloc_scratch(&base);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return nfail(nullptr, SF_ERR_HIP, "hipGetSymbolAddress of the scratch array failed: %s",
                     hipGetErrorString(e));
    }
    hipStream_t s = (hipStream_t)hip_stream;
    CnnSegs sg{};
    sg.n = 1;
    sg.base[0] = 0;
    sg.off[0] = 0;
    sg.rows[0] = rows;
    sg.cols[0] = cols;
    sg.total = (int)(((int64_t)rows * cols + 15) / 16 * 16);
    sg.base[1] = sg.total;
    sg.off[1] = rows * cols;
    uint16_t* act[2] = {(uint16_t*)(base + kNaAct0), (uint16_t*)(base + kNaAct1)};
    float* planes_in = (float*)(base + kNaIn);
    float* planes_out = (float*)(base + kNaOut);
    PackArgs p{};
    layer_offsets(p.woff, p.boff, p.cin, p.cout);
    p.params = params;
    p.wf = (uint16_t*)(base + kNaWf);
    p.wb = (uint16_t*)(base + kNaWb);
    p.bias = (float*)(base + kNaBias);
    e = launch_pack_weights(p, s);
    if (e == hipSuccess) e = launch_planes_in(sg, in, kCnnInputs, planes_in, s);
    if (e == hipSuccess) e = launch_pack_inputs(planes_in, kCnnInputs, sg.total, act[0], s);
    for (int l = 0; l < kCnnLayers && e == hipSuccess; ++l) {
        // one launch per layer (the sequence training runs; sf_net_forward's single launch
        // gives bitwise the same), activations ping-ponging between two buffers
        ConvArgs a{};
        a.segs = sg;
        a.in = act[l & 1];
        a.w = p.wf + (size_t)l * 9 * 256;
        a.bias = p.bias + l * 16;
        a.relu = l < kCnnLayers - 1;
        a.nout = l < kCnnLayers - 1 ? 16 : 3;
        a.out = l < kCnnLayers - 1 ? act[(l + 1) & 1] : nullptr;
        a.out_f32 = planes_out;
        e = launch_conv(a, l == kCnnLayers - 1, s);
    }
    if (e == hipSuccess) e = launch_planes_out(sg, planes_out, 3, out, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return nfail(nullptr, SF_ERR_HIP, "launching the forward pass failed: %s",
                     hipGetErrorString(e));
    }
    return SF_OK;
}

sf_status sf_net_set_loss(sf_net n, float eps) {
    sf_status st = net_alive(n);
    if (st != SF_OK) return st;
    if (!(eps > 0.0f) || !isfinite(eps)) return nfail(n, SF_ERR_INVALID_ARG, "eps must be finite and > 0");
    n->eps = eps;
    return SF_OK;
}

sf_status sf_net_destroy(sf_net n) {
    if (!n) return SF_OK;
    if (!n->hip_failed) (void)hipStreamSynchronize(n->stream);
    if (n->mem) (void)hipFree(n->mem);
    delete n;
    return SF_OK;
}

const char* sf_net_last_error(sf_net n) {
    return n ? n->err.c_str() : g_net_create_error;
}

}  // extern "C"
