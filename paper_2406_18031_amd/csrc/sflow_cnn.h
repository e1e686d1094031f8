// Structures and launchers of the learned update's network kernels (sflow_cnn.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sflow {

constexpr int kCnnMaxSegs = 64;
constexpr int kCnnLayers = 4;
constexpr int kCnnInputs = 9;
constexpr int kCnnParams = 6387;   // 9*16*9+16 + 2*(16*16*9+16) + 16*3*9+3

// A list of images stored one after the other; image k's pixels start at base[k] (a
// multiple of 16); total = padded end of the last image.
struct CnnSegs {
    int n;
    int total;
    int base[kCnnMaxSegs + 1];
    int off[kCnnMaxSegs + 1];    // unpadded pixel offset of image k (caller's packed layout)
    int rows[kCnnMaxSegs];
    int cols[kCnnMaxSegs];
};

struct ConvArgs {
    CnnSegs segs;
    const uint16_t* in;      // BF16 NHWC, 16 channels
    const uint16_t* mask;    // optional: keep input values only where mask > 0
    const uint16_t* w;       // BF16 [9][16 out][16 in]
    const float* bias;       // optional, 16
    int relu;
    int nout;                // meaningful output channels
    uint16_t* out;           // BF16 NHWC 16 channels (when not out_f32)
    float* out_f32;          // FP32 planes [nout][total] (when out_f32)
    int tblk[kCnnMaxSegs + 1];   // first block of each image's 16 x 16 tiles (set by launch_conv)
};

// The whole forward pass in one launch (k_net): input BF16 NHWC 16 (9 used), the packed
// forward weights and biases of the four layers, output FP32 planes [3][total].
struct NetArgs {
    CnnSegs segs;
    const uint16_t* in;
    const uint16_t* w;       // BF16 [4][9][16 out][16 in]
    const float* bias;       // FP32 [4][16]
    float* out_f32;
    int tblk[kCnnMaxSegs + 1];   // first block of each image's tiles (set by launch_net)
};

struct DwArgs {
    CnnSegs segs;
    const uint16_t* in;      // layer input, BF16 NHWC 16
    const uint16_t* dout;    // d loss / d layer output, BF16 NHWC 16
    const uint16_t* act;     // optional layer output (ReLU mask)
    int per_wave;            // 16-pixel groups reduced per wave
    float* dw;               // FP32 [9][16 in][16 out], accumulated
    float* db;               // FP32 [16], accumulated
};

struct LossArgs {
    CnnSegs segs;
    const float* out;        // FP32 planes [3][total]
    const float* target;     // FP32 planes [3][total]
    float eps, inv_count;
    float* loss;             // accumulated
    uint16_t* dout;          // BF16 NHWC 16
};

struct AdamArgs {
    float* params;
    const float* grad;
    float* m;
    float* v;
    int nparams;
    float lr, b1, b2, eps, c1, c2;
};

struct PackArgs {
    const float* params;     // FP32 master, per layer W (3, 3, cin, cout) then b (cout)
    int woff[kCnnLayers], boff[kCnnLayers], cin[kCnnLayers], cout[kCnnLayers];
    uint16_t* wf;            // BF16 [4][9][16][16] forward weights
    uint16_t* wb;            // BF16 [4][9][16][16] input-gradient weights
    float* bias;             // FP32 [4][16]
};

// gradient of the FP32 master parameters from the per-layer [9][16][16] / [16] sums
struct GradArgs {
    int woff[kCnnLayers], boff[kCnnLayers], cin[kCnnLayers], cout[kCnnLayers];
    const float* dw;         // FP32 [4][9][16 in][16 out]
    const float* db;         // FP32 [4][16]
    float* grad;             // FP32 [kCnnParams]
};

hipError_t launch_conv(const ConvArgs& a, bool out_f32, hipStream_t s);
hipError_t launch_net(const NetArgs& a, hipStream_t s);
hipError_t launch_conv_dw(const DwArgs& a, hipStream_t s);
hipError_t launch_loss(const LossArgs& a, hipStream_t s);
hipError_t launch_pack_inputs(const float* in, int C, int total, uint16_t* out, hipStream_t s);
hipError_t launch_adam(const AdamArgs& a, hipStream_t s);
hipError_t launch_pack_weights(const PackArgs& a, hipStream_t s);
hipError_t launch_gather_grads(const GradArgs& a, hipStream_t s);
// caller layout (images one after the other, each [C][rows][cols]) <-> padded planes [C][total]
hipError_t launch_planes_in(const CnnSegs& sg, const float* src, int C, float* dst, hipStream_t s);
hipError_t launch_planes_out(const CnnSegs& sg, const float* src, int C, float* dst, hipStream_t s);

}  // namespace sflow
