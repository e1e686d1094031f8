// Internal structures shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sflow.h"
#include "sflow_cnn.h"

namespace sflow {

constexpr int kMaxLevels = SF_MAX_LEVELS;
constexpr int kBlock = 1024;         // threads per block of the fused level kernel
constexpr int kRegion = 64;          // max rows/columns of a tile plus its halo
// LDS of the fused level kernel: the larger of the row-pass exchange buffers
// (2 buffers x waves x 2 rows x 8 fields x 64 lanes) and the update planes (8 x 64 x 64: the
// image model's 2, the smoothing's 2 x 3)
constexpr size_t kLdsXB = 2 * (kBlock / 64) * 2 * 8 * 64 * sizeof(float);
constexpr size_t kLdsPlanes = 8 * kRegion * 64 * sizeof(float);
constexpr size_t kLdsBytes = kLdsXB > kLdsPlanes ? kLdsXB : kLdsPlanes;

constexpr int kMaxStreams = 64;        // camera streams per context
constexpr int kLevelPad = 2;           // zeroed entries after the device level table
constexpr int kDefaultPassSteps = 8;   // prediction steps per step launch before a level splits
// FP32 -> BF16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Planes of the learned-update buffers of a finest level, each `ltotal` floats: 9 unused (the
// network's 9 inputs go to `lpack`, BF16), prior x0 (3), least-squares solution (3), cost terms
// a_Y (3), a_rho (3), G1, G2 (2), 3 unused (the network's output stays in LDS: the network and
// the choice run in one launch), the smoothed solution (3) and the applied correction (3).
constexpr int kLearnInputs = 9;
constexpr int kLearnX0 = 9, kLearnXP = 12, kLearnFB = 15, kLearnOut = 23;
constexpr int kLearnXS = 26;      // smoothed least-squares solution (the state)
constexpr int kLearnCorr = 29;    // applied correction, rad/frame (0 where it fell back)
constexpr int kLearnPlanes = 32;
constexpr int kElemBlock = 256;      // threads (pixels) per block of the per-pixel kernels
constexpr int kTile2 = 16;           // tile side of the two-level pyramid / reconstruction kernels
static_assert(kTile2 * kTile2 == kElemBlock, "one thread per tile pixel");

// Parameters of one pyramid level of one camera stream ("entry"), uploaded to device memory
// whenever the camera or the tiling changes.  Entries are ordered stream by stream, finest
// level first, so a level's finer and coarser neighbours are entries e - 1 and e + 1.  The
// device table is followed by kLevelPad zeroed entries: kernels read entries e + 1 and e + 2
// before knowing whether they belong to the same stream.
struct LevelDev {
    int rows, cols, pitch;           // level size; row pitch (elements) of state/pyramid planes
    float ifx, ify, cxn, cyn;        // x = j*ifx - cxn, y = i*ify - cyn (pinhole ray)
    float fx;
    int N, Ns, top;                  // prediction steps, smoothing passes, 1 = coarsest level
    float g1, g2, g3, g4, g5;        // gamma_1..gamma_5
    float qscale;                    // half storage: stored flow = flow (rad/frame) * qscale
    int tw, th, tiles_x, tiles_y, block0, halo;
    int stream, level;               // owning stream; level (0 = finest)
    int child, parent;               // entries of the next finer / coarser level (-1: none)
    uint32_t flags;                  // SF_READ_* bits of the stream
    int learned;                     // 1: the update of this level is the learned one
    int lbase;                       // first pixel of this level in the learned buffers
    int ltotal;                      // pixels (padded) of the learned buffers, all streams
    float* lbuf;                     // learned buffers: kLearnPlanes planes of ltotal floats
    uint16_t* lpack;                 // the network's input: BF16, 16 channels per pixel (9 used)
    void* w[2][3];                   // state, indexed by parity
    void* dw[2][3];                  // lower levels only
    void* rho[2];
    void* Y[2];
    void* Ym[2];                     // pyramid image of a frame (levels >= 1), two buffers
    void* Rm[2];                     // pyramid inverse depth, the same (FrameInputs::mbuf)
    // The prediction of a level may be split over several step launches ("passes") of at most
    // a few steps each, so that each pass needs a smaller halo.  A pass entry is a copy of its
    // level's entry with its own halo and tiles, and:
    // General grids of directions: 9 planes of rows x gpitch floats (b1/dmu (3), b2/dmu (3),
    // eta (3)), or NULL for the pinhole grid of the intrinsics above
    const float* geo;
    int gpitch;
    int pass_n;                      // steps of this pass (N, the level's steps, sets dt)
    int pass_first;                  // 1: loads the frame-k state (and applies the dt rescale)
    int pass_last;                   // 1: runs the update, smoothing and state store
    float* mid_in[8];                // FP32 fields after the previous pass (pitch = pitch)
    float* mid_out[8];               // FP32 fields after this pass
    // the context's watchdog word: the kernels that store a level's new flow set bit `stream`
    // when a value is not finite (or, in FP16 storage, beyond its range); sf_check_state reads
    // and clears it
    unsigned long long* numeric;
};

// Per-frame arguments: the finest-level measurements of every stream (caller's device
// pointers, pitch = cols), the dt_new / dt_old rescale of w and dw, and which of the two
// pyramid buffers the frame's pyramid is written to and read from (consecutive frames
// alternate, so that a frame's pyramid can be built while the previous frame's level step
// still reads its own).
struct FrameInputs {
    const void* Y[kMaxStreams];
    const void* R[kMaxStreams];
    float scale[kMaxStreams];
    int mbuf;
};

// Camera rates of one stream for the inertial source terms of the prediction, in the filter's
// time unit: angular velocity Omega (rad/frame), its rate of change dOmega (rad/frame^2) and
// linear acceleration a (1/frame^2; times an inverse depth it is a structure-flow rate
// change), all in the camera frame.
struct Inertial {
    float ox, oy, oz, dx, dy, dz, ax, ay, az;
};

struct StepArgs {
    const LevelDev* lv;              // the pass entries of this launch
    int nent;                        // entries; entry e owns blocks [lv[e].block0, lv[e+1].block0)
    int parity;                      // state[parity] is frame k, state[1 - parity] receives k+1
    FrameInputs in;
    Inertial imu[kMaxStreams];       // read by the inertial form of the kernel only
};

// A launch of a per-pixel kernel over a list of entries: entry ent[k] owns blocks
// [blk[k], blk[k+1]) of kElemBlock pixels each (for the pyramid and reconstruction kernels: of
// tiles of the side the launch is made with, kTile2 or 2 kTile2).
struct ElemArgs {
    const LevelDev* lv;
    int n;
    int ent[kMaxStreams];
    int blk[kMaxStreams + 1];
    int parity;                      // state parity read/written by the kernel
    int kind;                        // output kind (k_output, k_reconstruct)
    float* out;                      // output planes (k_learned_extract)
    float* outs[kMaxStreams];        // k_output, k_reconstruct: output planes of the launch's
                                     // k-th entry (NULL: none)
    float inv_dts[kMaxStreams];      // their scale to rad/s
    FrameInputs in;
};

// Mapping of a pinhole camera's frame onto the finest grid of a stream (k_map): one thread per
// grid pixel of entry `ent`.
struct MapArgs {
    const LevelDev* lv;
    int ent;
    float fx, fy, cx, cy;            // the source camera
    int rows, cols;                  // its size
    const void* Y;                   // source image and inverse depth (storage type, rows x cols)
    const void* R;
    void* Yout;                      // grid image and inverse depth (storage type, level size)
    void* Rout;
};
hipError_t launch_map(int storage, const MapArgs& a, int pixels, hipStream_t s);

// Inverse depth from a rectified stereo pair (k_stereo, sflow_stereo.hip): one thread per pixel
// of the stream's finest level.
struct StereoArgs {
    const void* YL;                  // left (the filter's) and right images, storage type
    const void* YR;
    void* rho;                       // inverse-depth measurement out, storage type
    int rows, cols;
    float fx, fy, cx, cy;            // left pinhole camera
    float baseline;                  // metres along the left camera's x axis
    int dmax, iters;                 // search range [0, dmax] px, Gauss-Newton steps
    float texture, residual;         // validity thresholds
};
hipError_t launch_stereo(int storage, const StereoArgs& a, hipStream_t s);

// Device allocation of the library (hipMalloc, with a failure-injection hook for tests: the
// environment variable SFLOW_FAIL_ALLOC=n fails the n-th allocation counted from the moment
// the variable took its current value).
hipError_t dev_malloc(void** p, size_t bytes);

// kernel launchers (sflow_kernels.hip); `storage` is SF_FP32 or SF_FP16
// tile: kTile2 or 2 kTile2 (the blocks in a.blk count tiles of that size)
hipError_t launch_pyramid(int storage, int tile, const ElemArgs& a, hipStream_t s);
hipError_t launch_init(int storage, const ElemArgs& a, hipStream_t s);
// inertial: the prediction keeps the inertial source terms with the rates in a.imu;
// grid: the levels' geometry comes from their tables (LevelDev::geo), not the pinhole
hipError_t launch_step(int storage, bool inertial, bool grid, const StepArgs& a, int nblocks,
                       size_t lds_bytes, hipStream_t s);
// tile: kTile2 (one level-h pixel per thread) or 2 kTile2 (four); the blocks in a.blk count
// tiles of that size
hipError_t launch_reconstruct(int storage, int tile, const ElemArgs& a, hipStream_t s);
hipError_t launch_output(int storage, const ElemArgs& a, hipStream_t s);
hipError_t launch_learned_extract(int storage, const ElemArgs& a, hipStream_t s);
hipError_t prepare_kernels(size_t max_lds_bytes);
// Which per-frame arguments a kernel of this library reads, for updating the kernel nodes of a
// captured frame graph: 1 = ElemArgs::in (the pyramid), 2 = StepArgs::in and ::imu (the level
// step), 0 = none (the other kernels' arguments do not change from frame to frame).
int frame_input_kind(const void* func);

// learned update, one launch for all streams: the network on every stream's finest level
// (net: its images are the streams' finest levels, in stream order), then the choice between
// the network's and the least-squares solution per pixel, the smoothing and the store of the
// finest level's new flow state
struct NetCombineArgs {
    NetArgs net;
    const LevelDev* lv;
    int ent[kMaxStreams];            // the finest level's entry of image k
    int parity;                      // state parity written
    float threshold;                 // fallback when the cost increase exceeds it
    unsigned long long* fallbacks;   // accumulated count of pixels that fell back
};
hipError_t launch_net_combine(int storage, const NetCombineArgs& a, hipStream_t s);

}  // namespace sflow
