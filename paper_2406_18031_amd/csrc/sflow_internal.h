// Internal structures shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sflow.h"

namespace sflow {

constexpr int kMaxLevels = SF_MAX_LEVELS;
constexpr int kBlock = 1024;         // threads per block of the fused level kernel
constexpr int kRegion = 64;          // max rows/columns of a tile plus its halo
// LDS of the fused level kernel: the larger of the row-pass exchange buffers
// (2 buffers x waves x 2 rows x 8 fields x 64 lanes) and the update planes (5 x 64 x 64)
constexpr size_t kLdsXB = 2 * (kBlock / 64) * 2 * 8 * 64 * sizeof(float);
constexpr size_t kLdsPlanes = 5 * kRegion * 64 * sizeof(float);
constexpr size_t kLdsBytes = kLdsXB > kLdsPlanes ? kLdsXB : kLdsPlanes;

// Per-level parameters, uploaded once per camera to device memory.
struct LevelDev {
    int rows, cols, pitch;           // level size; row pitch (elements) of state/pyramid planes
    float ifx, ify, cxn, cyn;        // x = j*ifx - cxn, y = i*ify - cyn (pinhole ray)
    float fx;
    int N, Ns, top;                  // prediction steps, smoothing passes, 1 = coarsest level
    float g1, g2, g3, g4, g5;        // gamma_1..gamma_5
    float qscale;                    // half storage: stored flow = flow (rad/frame) * qscale
    int tw, th, tiles_x, tiles_y, block0, halo;
    void* w[2][3];                   // state, indexed by parity
    void* dw[2][3];                  // lower levels only
    void* rho[2];
    void* Y[2];
    void* Ym;                        // pyramid image of this frame (levels >= 2)
    void* Rm;                        // pyramid inverse depth of this frame (levels >= 2)
};

struct StepArgs {
    const LevelDev* lv;
    int nlev;
    const void* Y1;                  // finest-level measurements of this frame (pitch = cols)
    const void* R1;
    int parity;                      // state[parity] is frame k, state[1 - parity] receives k+1
    float scale;                     // dt_new / dt_old rescale of w and dw (1 when unchanged)
    uint32_t flags;                  // SF_READ_* bits
};

// kernel launchers (sflow_kernels.hip)
hipError_t launch_pyramid(int storage, const LevelDev* lv_host, const LevelDev* lv_dev, int h,
                          const void* Ysrc, const void* Rsrc, int src_pitch, hipStream_t s);
hipError_t launch_init(int storage, const LevelDev* lv_host, const LevelDev* lv_dev, int h,
                       const void* Ym, const void* Rm, int meas_pitch, hipStream_t s);
hipError_t launch_step(int storage, const StepArgs& a, int nblocks, size_t lds_bytes,
                       hipStream_t s);
hipError_t launch_reconstruct(int storage, const LevelDev* lv_host, const LevelDev* lv_dev,
                              int h, int parity_out, hipStream_t s);
hipError_t launch_output(int storage, const LevelDev* lv_host, const LevelDev* lv_dev,
                         int parity, int kind, float inv_dt, float* out, hipStream_t s);
hipError_t prepare_kernels(size_t max_lds_bytes);

}  // namespace sflow
