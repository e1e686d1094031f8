// Exercises the library's C ABI end to end under AddressSanitizer: the host code (runtime, C ABI
// and this driver) is instrumented, the device code is the product's.  Every call's status is
// checked against the one it must return, the error paths included.  Built, together with the
// library's sources into one executable (the sanitizer runtime linked in, nothing to preload),
// by `python -m paper_2406_18031_amd.build --asan`; exit status 0 when every check held.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "sflow.h"

static int g_checks = 0, g_fail = 0;
#define EXPECT(call, want)                                                                  \
    do {                                                                                    \
        const sf_status s_ = (call);                                                        \
        ++g_checks;                                                                         \
        if (s_ != (want)) {                                                                 \
            printf("FAIL line %d: %s -> %d, expected %d\n", __LINE__, #call, (int)s_,      \
                   (int)(want));                                                            \
            ++g_fail;                                                                       \
        }                                                                                   \
    } while (0)

static std::vector<void*> g_dev;
static void* dev_bytes(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, n) != hipSuccess) return nullptr;
    (void)hipMemset(p, 0, n);
    g_dev.push_back(p);
    return p;
}
static void* upload_f32(const std::vector<float>& h) {
    void* p = dev_bytes(h.size() * sizeof(float));
    if (p) (void)hipMemcpy(p, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice);
    return p;
}
static void* upload_f16(const std::vector<float>& h) {
    std::vector<__half> v(h.size());
    for (size_t i = 0; i < h.size(); ++i) v[i] = __float2half(h[i]);
    void* p = dev_bytes(v.size() * sizeof(__half));
    if (p) (void)hipMemcpy(p, v.data(), v.size() * sizeof(__half), hipMemcpyHostToDevice);
    return p;
}

// frame k of a moving texture: brightness in [0, 1], inverse depth in [0.2, 0.5] with 5 % missing
static void frame(int R, int C, int k, std::vector<float>& Y, std::vector<float>& rho) {
    std::mt19937 g(1234u + (unsigned)k);
    std::uniform_real_distribution<float> u(0.0f, 1.0f);
    Y.resize((size_t)R * C);
    rho.resize((size_t)R * C);
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < C; ++j) {
            const float x = 0.21f * (j + 0.7f * k), y = 0.17f * (i + 0.3f * k);
            Y[(size_t)i * C + j] = 0.5f + 0.25f * std::sin(x) * std::cos(y) + 0.1f * u(g);
            const float r = 0.2f + 0.3f * u(g);
            rho[(size_t)i * C + j] = u(g) < 0.05f ? NAN : r;
        }
}

static sf_config config(int R, int C, int H, float mf, int storage, int update) {
    sf_config c;
    memset(&c, 0, sizeof c);
    c.rows = R;
    c.cols = C;
    c.levels = H;
    c.max_flow_px = mf;
    for (int h = 0; h < H; ++h) c.smooth_iters[h] = h == 0 ? 2 : 4;
    c.storage = storage;
    c.update = update;
    return c;
}

static sf_camera pinhole(int R, int C) {
    sf_camera cam;
    memset(&cam, 0, sizeof cam);
    cam.fx = cam.fy = 0.9 * C;
    cam.cx = 0.5 * (C - 1);
    cam.cy = 0.5 * (R - 1);
    return cam;
}

static void single_stream(int storage) {
    const int R = 96, C = 128;
    const size_t px = (size_t)R * C;
    sf_config cfg = config(R, C, 3, 4.0f, storage, SF_UPDATE_PLAIN);
    sf_ctx c = nullptr;
    EXPECT(sf_create(&cfg, nullptr, &c), SF_OK);
    if (!c) return;
    std::vector<float> Y, rho;
    std::vector<void*> dY, dR;
    for (int k = 0; k < 8; ++k) {
        frame(R, C, k, Y, rho);
        dY.push_back(storage == SF_FP16 ? upload_f16(Y) : upload_f32(Y));
        dR.push_back(storage == SF_FP16 ? upload_f16(rho) : upload_f32(rho));
    }
    float* out = (float*)dev_bytes(3 * px * sizeof(float));
    EXPECT(sf_push_frame(c, dY[0], dR[0], 0.01), SF_ERR_STATE);   // no camera yet
    const sf_camera cam = pinhole(R, C);
    EXPECT(sf_set_camera(c, &cam), SF_OK);
    EXPECT(sf_get_flow(c, SF_FLOW_W_FRAME, out), SF_ERR_STATE);    // no push yet
    EXPECT(sf_push_frame(c, Y.data(), rho.data(), 0.01), SF_ERR_INVALID_ARG);   // host pointers
    EXPECT(sf_push_frame(c, dY[0], dR[0], 0.0), SF_ERR_INVALID_ARG);
    EXPECT(sf_push_frame(c, dY[0], dR[0], NAN), SF_ERR_INVALID_ARG);
    for (int k = 0; k < 4; ++k) EXPECT(sf_push_frame(c, dY[k], dR[k], 0.01), SF_OK);
    for (int kind = 0; kind <= 4; ++kind) EXPECT(sf_get_flow(c, kind, out), SF_OK);
    EXPECT(sf_get_flow(c, 5, out), SF_ERR_INVALID_ARG);
    EXPECT(sf_get_flow(c, SF_FLOW_W_FRAME, nullptr), SF_ERR_INVALID_ARG);
    const double om[3] = {0.01, -0.02, 0.005}, dom[3] = {0.0, 0.001, 0.0}, acc[3] = {0.1, 0.0, 0.0};
    EXPECT(sf_push_frame_ex(c, dY[4], dR[4], 0.01, om, dom, acc), SF_OK);
    const double bad[3] = {NAN, 0.0, 0.0};
    EXPECT(sf_push_frame_ex(c, dY[4], dR[4], 0.01, bad, nullptr, nullptr), SF_ERR_INVALID_ARG);
    size_t n = 0;
    EXPECT(sf_state_size(c, &n), SF_OK);
    std::vector<unsigned char> blob(n);
    EXPECT(sf_get_state(c, blob.data(), n), SF_OK);
    EXPECT(sf_get_state(c, blob.data(), n - 1), SF_ERR_INVALID_ARG);
    EXPECT(sf_set_state(c, blob.data(), n), SF_OK);
    EXPECT(sf_set_state(c, blob.data(), n + 1), SF_ERR_INVALID_ARG);
    EXPECT(sf_set_tile(c, 1, 40, 40), SF_OK);
    EXPECT(sf_set_tile(c, 0, 40, 40), SF_ERR_INVALID_ARG);   // levels count from 1
    EXPECT(sf_set_tile(c, 9, 40, 40), SF_ERR_INVALID_ARG);
    EXPECT(sf_push_frame(c, dY[5], dR[5], 0.01), SF_OK);
    EXPECT(sf_set_pass_steps(c, 2), SF_OK);
    EXPECT(sf_push_frame(c, dY[6], dR[6], 0.02), SF_OK);
    EXPECT(sf_set_pass_steps(c, 0), SF_ERR_INVALID_ARG);
    EXPECT(sf_set_pass_steps(c, 64), SF_OK);                 // one pass per level again
    EXPECT(sf_set_timing(c, 1), SF_OK);
    EXPECT(sf_push_frame(c, dY[7], dR[7], 0.01), SF_OK);
    double ms[3];
    int64_t launches[3];
    EXPECT(sf_kernel_times(c, ms, launches, 1), SF_OK);
    EXPECT(sf_set_timing(c, 0), SF_OK);
    EXPECT(sf_set_graph(c, 1), SF_OK);
    for (int k = 0; k < 4; ++k) {
        EXPECT(sf_push_frame(c, dY[k], dR[k], 0.01), SF_OK);
        EXPECT(sf_get_flow(c, SF_FLOW_W_RAD_S, out), SF_OK);
    }
    EXPECT(sf_set_graph(c, 0), SF_OK);
    hipStream_t in_stream = nullptr;
    (void)hipStreamCreate(&in_stream);
    EXPECT(sf_set_input_stream(c, in_stream), SF_OK);
    for (int k = 4; k < 8; ++k) EXPECT(sf_push_frame(c, dY[k], dR[k], 0.01), SF_OK);
    EXPECT(sf_set_input_stream(c, nullptr), SF_OK);
    (void)hipStreamSynchronize(in_stream);
    (void)hipStreamDestroy(in_stream);
    uint64_t mask = 1;
    EXPECT(sf_check_state(c, &mask), SF_OK);
    EXPECT(sf_check_state(c, nullptr), SF_ERR_INVALID_ARG);
    float* upd = (float*)dev_bytes(SF_UPDATE_INPUT_PLANES * px * sizeof(float));
    EXPECT(sf_get_update_inputs(c, 0, upd), SF_ERR_STATE);          // not a learned context
    EXPECT(sf_set_learned(c, nullptr, 0, 0.5f), SF_ERR_STATE);         // not a learned context
    int32_t ns = 0;
    EXPECT(sf_stream_count(c, &ns), SF_OK);
    if (!sf_last_error(c)) ++g_fail;
    EXPECT(sf_destroy(c), SF_OK);
}

static void batch() {
    const int sizes[3][2] = {{96, 128}, {70, 60}, {40, 40}};
    const int levels[3] = {3, 2, 1};
    sf_config cfg[3];
    sf_camera cams[3];
    for (int s = 0; s < 3; ++s) {
        cfg[s] = config(sizes[s][0], sizes[s][1], levels[s], 3.0f, SF_FP32, SF_UPDATE_PLAIN);
        cams[s] = pinhole(sizes[s][0], sizes[s][1]);
    }
    sf_ctx c = nullptr;
    EXPECT(sf_create_batch(cfg, 0, nullptr, &c), SF_ERR_INVALID_ARG);
    EXPECT(sf_create_batch(cfg, 3, nullptr, &c), SF_OK);
    if (!c) return;
    EXPECT(sf_set_cameras(c, cams), SF_OK);
    const void* Yp[3];
    const void* Rp[3];
    void* outs[3];
    std::vector<float> Y, rho;
    for (int k = 0; k < 4; ++k) {
        for (int s = 0; s < 3; ++s) {
            frame(sizes[s][0], sizes[s][1], k, Y, rho);
            Yp[s] = upload_f32(Y);
            Rp[s] = upload_f32(rho);
            outs[s] = dev_bytes(3 * (size_t)sizes[s][0] * sizes[s][1] * sizeof(float));
        }
        const double dts[3] = {0.01, 0.01, 0.02};
        EXPECT(sf_push_frames(c, Yp, Rp, dts), SF_OK);
        EXPECT(sf_get_flows(c, SF_FLOW_W_FRAME, outs), SF_OK);
    }
    EXPECT(sf_get_flow_stream(c, 2, SF_FLOW_RHO, outs[2]), SF_OK);
    EXPECT(sf_get_flow_stream(c, 3, SF_FLOW_RHO, outs[2]), SF_ERR_INVALID_ARG);
    EXPECT(sf_push_frame(c, Yp[0], Rp[0], 0.01), SF_ERR_INVALID_ARG);   // a batch takes frames
    for (int s = 0; s < 3; ++s) {
        size_t n = 0;
        EXPECT(sf_state_size_stream(c, s, &n), SF_OK);
        std::vector<unsigned char> blob(n);
        EXPECT(sf_get_state_stream(c, s, blob.data(), n), SF_OK);
        EXPECT(sf_set_state_stream(c, s, blob.data(), n), SF_OK);
    }
    uint64_t mask = 1;
    EXPECT(sf_check_state(c, &mask), SF_OK);
    EXPECT(sf_destroy(c), SF_OK);
}

static void learned() {
    const int R = 64, C = 96;
    const size_t px = (size_t)R * C;
    sf_config cfg = config(R, C, 2, 3.0f, SF_FP32, SF_UPDATE_LEARNED);
    sf_ctx c = nullptr;
    EXPECT(sf_create(&cfg, nullptr, &c), SF_OK);
    if (!c) return;
    const sf_camera cam = pinhole(R, C);
    EXPECT(sf_set_camera(c, &cam), SF_OK);
    std::vector<float> Y, rho;
    frame(R, C, 0, Y, rho);
    void* dY = upload_f32(Y);
    void* dR = upload_f32(rho);
    EXPECT(sf_push_frame(c, dY, dR, 0.01), SF_ERR_STATE);   // parameters first
    std::vector<float> p(SF_LEARNED_PARAMS);
    std::mt19937 g(7);
    std::normal_distribution<float> nd(0.0f, 0.05f);
    for (auto& v : p) v = nd(g);
    EXPECT(sf_set_learned(c, p.data(), p.size() - 1, 0.5f), SF_ERR_INVALID_ARG);
    EXPECT(sf_set_learned(c, p.data(), p.size(), 0.5f), SF_OK);
    for (int k = 0; k < 4; ++k) {
        frame(R, C, k, Y, rho);
        EXPECT(sf_push_frame(c, upload_f32(Y), upload_f32(rho), 0.01), SF_OK);
    }
    int64_t fb = 0, pix = 0;
    EXPECT(sf_learned_stats(c, &fb, &pix, 1), SF_OK);
    float* upd = (float*)dev_bytes(SF_UPDATE_INPUT_PLANES * px * sizeof(float));
    EXPECT(sf_get_update_inputs(c, 0, upd), SF_OK);
    float* out = (float*)dev_bytes(3 * px * sizeof(float));
    EXPECT(sf_get_flow(c, SF_FLOW_W_RAD_S, out), SF_OK);
    EXPECT(sf_destroy(c), SF_OK);
}

static void grid_mapping_stereo() {
    const int R = 64, C = 80, SR = 80, SC = 100;
    std::vector<double> eta((size_t)R * C * 3);
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < C; ++j) {
            const double lon = (j - 0.5 * (C - 1)) * 0.012, lat = (i - 0.5 * (R - 1)) * 0.012;
            double* e = &eta[((size_t)i * C + j) * 3];
            e[0] = std::cos(lat) * std::sin(lon);
            e[1] = std::sin(lat);
            e[2] = std::cos(lat) * std::cos(lon);
        }
    sf_config cfg = config(R, C, 2, 3.0f, SF_FP32, SF_UPDATE_PLAIN);
    sf_ctx c = nullptr;
    EXPECT(sf_create(&cfg, nullptr, &c), SF_OK);
    if (!c) return;
    sf_camera cam = pinhole(R, C);
    cam.eta = eta.data();
    EXPECT(sf_set_camera(c, &cam), SF_OK);
    sf_camera src = pinhole(SR, SC);
    EXPECT(sf_set_source_camera(c, 0, &src, SR, SC), SF_OK);
    std::vector<float> Y, rho;
    void* Yo = dev_bytes((size_t)R * C * sizeof(float));
    void* Ro = dev_bytes((size_t)R * C * sizeof(float));
    for (int k = 0; k < 3; ++k) {
        frame(SR, SC, k, Y, rho);
        EXPECT(sf_map_frame(c, 0, upload_f32(Y), upload_f32(rho), Yo, Ro), SF_OK);
        EXPECT(sf_push_frame(c, Yo, Ro, 0.01), SF_OK);
    }
    EXPECT(sf_set_stereo(c, 0, 0.1, 16, 3, 2.5e-3, 0.05), SF_OK);
    EXPECT(sf_stereo_depth(c, 0, Yo, Yo, Ro), SF_ERR_UNSUPPORTED);   // a grid stream
    EXPECT(sf_destroy(c), SF_OK);
    // stereo on a pinhole stream
    EXPECT(sf_create(&cfg, nullptr, &c), SF_OK);
    if (!c) return;
    const sf_camera pin = pinhole(R, C);
    EXPECT(sf_set_camera(c, &pin), SF_OK);
    EXPECT(sf_set_stereo(c, 0, -1.0, 16, 3, 2.5e-3, 0.05), SF_ERR_INVALID_ARG);
    EXPECT(sf_set_stereo(c, 0, 0.1, 16, 3, 2.5e-3, 0.05), SF_OK);
    for (int k = 0; k < 3; ++k) {
        frame(R, C, k, Y, rho);
        void* L = upload_f32(Y);
        frame(R, C, k + 1, Y, rho);
        void* Rt = upload_f32(Y);
        EXPECT(sf_stereo_depth(c, 0, L, Rt, Ro), SF_OK);
        EXPECT(sf_push_frame(c, L, Ro, 0.01), SF_OK);
    }
    EXPECT(sf_destroy(c), SF_OK);
}

static void network() {
    const int32_t rows[2] = {40, 24}, cols[2] = {56, 33};
    size_t px = 0;
    for (int k = 0; k < 2; ++k) px += (size_t)rows[k] * cols[k];
    sf_net net = nullptr;
    EXPECT(sf_net_create(rows, cols, 0, nullptr, &net), SF_ERR_INVALID_ARG);
    EXPECT(sf_net_create(rows, cols, 2, nullptr, &net), SF_OK);
    if (!net) return;
    std::vector<float> p(SF_LEARNED_PARAMS), q(SF_LEARNED_PARAMS), grad(SF_LEARNED_PARAMS);
    std::mt19937 g(11);
    std::normal_distribution<float> nd(0.0f, 0.05f);
    for (auto& v : p) v = nd(g);
    EXPECT(sf_net_set_params(net, p.data(), p.size()), SF_OK);
    EXPECT(sf_net_get_params(net, q.data(), q.size()), SF_OK);
    if (memcmp(p.data(), q.data(), p.size() * sizeof(float)) != 0) ++g_fail;
    std::vector<float> in(9 * px), tgt(3 * px);
    for (auto& v : in) v = nd(g);
    for (auto& v : tgt) v = nd(g);
    float* din = (float*)upload_f32(in);
    float* dt = (float*)upload_f32(tgt);
    float* dout = (float*)dev_bytes(3 * px * sizeof(float));
    EXPECT(sf_net_forward(net, din, dout), SF_OK);
    EXPECT(sf_net_set_loss(net, 0.5f), SF_OK);
    EXPECT(sf_net_set_loss(net, -1.0f), SF_ERR_INVALID_ARG);
    float loss = 0.0f;
    EXPECT(sf_net_train_step(net, din, dt, 1e-3f, &loss, grad.data()), SF_OK);
    EXPECT(sf_net_train_step(net, din, dt, 0.0f, nullptr, nullptr), SF_OK);
    EXPECT(sf_net_destroy(net), SF_OK);
    EXPECT(sf_net_destroy(nullptr), SF_OK);
    float* dp = (float*)upload_f32(p);
    EXPECT(sf_net_forward_noalloc(dp, rows[0], cols[0], din, dout, nullptr), SF_OK);
    EXPECT(sf_net_forward_noalloc(dp, 0, cols[0], din, dout, nullptr), SF_ERR_INVALID_ARG);
    EXPECT(sf_net_forward_noalloc(p.data(), rows[0], cols[0], din, dout, nullptr),
           SF_ERR_INVALID_ARG);   // host parameters
    (void)hipDeviceSynchronize();
}

int main() {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        printf("abi driver: no GPU\n");
        return 2;
    }
    sf_config bad = config(1, 128, 1, 1.0f, SF_FP32, SF_UPDATE_PLAIN);
    sf_ctx c = nullptr;
    EXPECT(sf_create(&bad, nullptr, &c), SF_ERR_INVALID_ARG);
    EXPECT(sf_create(nullptr, nullptr, &c), SF_ERR_INVALID_ARG);
    bad = config(64, 64, SF_MAX_LEVELS + 1, 1.0f, SF_FP32, SF_UPDATE_PLAIN);
    EXPECT(sf_create(&bad, nullptr, &c), SF_ERR_INVALID_ARG);
    if (!sf_last_error(nullptr)) ++g_fail;
    single_stream(SF_FP32);
    single_stream(SF_FP16);
    batch();
    learned();
    grid_mapping_stereo();
    network();
    void* a = dev_bytes(1 << 20);
    void* b = dev_bytes(1 << 20);
    EXPECT(sf_copy_probe(a, b, 1 << 20, nullptr), SF_OK);
    (void)hipDeviceSynchronize();
    for (void* p : g_dev) (void)hipFree(p);
    printf("abi driver: %d checks, %d failed\n", g_checks, g_fail);
    return g_fail ? 1 : 0;
}
