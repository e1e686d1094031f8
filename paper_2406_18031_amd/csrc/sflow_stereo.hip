// Inverse depth from a rectified stereo pair on gfx950 (sf_stereo_depth in include/sflow.h):
// the paper's proposed extension (Section "Conclusions and Future Work") of taking the depth
// measurements from image disparity so that the update runs on image data only.
//
// Left camera = the stream's pinhole camera; the right camera has the same intrinsics and
// orientation, its centre `baseline` metres along the left camera's x axis, so a point at
// inverse range rho along the left direction eta appears d = kappa rho pixels to the left on the
// same row, kappa = fx baseline sqrt(x^2 + y^2 + 1), x = (j - cx)/fx, y = (i - cy)/fy.
// Per pixel: block matching over integer d in [0, D] (sum of absolute differences over a 5x5
// window, rows and columns clamped to the image, float32 sums over window rows then columns,
// the smallest d on ties), a few Gauss-Newton steps on the window's squared residuals with the
// right image interpolated linearly along the row, and rho = d / kappa, missing (NaN) where the
// window has too little texture along the row, the match is poor, or the point leaves the
// right image.
//
// A block computes a 16 x 16 tile.  It stages the left image over the tile's window
// (20 x 20) and the right image over every column the search and the refinement can reach
// (20 x (22 + D)) in LDS, each value at its clamped image position, so the window sums read
// exactly the clamped samples the definition names.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sflow_internal.h"

namespace sflow {
namespace {

__device__ __forceinline__ float sld(const float* p, size_t i) { return p[i]; }
__device__ __forceinline__ float sld(const __half* p, size_t i) { return __half2float(p[i]); }
__device__ __forceinline__ void sst(float* p, size_t i, float v) { p[i] = v; }
__device__ __forceinline__ void sst(__half* p, size_t i, float v) { p[i] = __float2half(v); }

constexpr int kT = 16;              // tile side
constexpr int kW = 2;               // window radius
constexpr int kMaxD = 64;           // largest disparity searched
constexpr int kLW = kT + 2 * kW;    // staged left tile side (20)
constexpr int kRW = kLW + 2 + kMaxD;  // staged right tile width, at most

__device__ __forceinline__ int clampi_s(int v, int lo, int hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

template <typename T>
__global__ void __launch_bounds__(kT * kT) k_stereo(StereoArgs a) {
    __shared__ float L[kLW][kLW];
    __shared__ float Rt[kLW][kRW];
    const int tiles_x = (a.cols + kT - 1) / kT;
    const int ti0 = (blockIdx.x / tiles_x) * kT, tj0 = (blockIdx.x % tiles_x) * kT;
    const int D = a.dmax;
    const int rw = kLW + 2 + D;            // staged right width for this search range
    const int rbase = tj0 - kW - D - 1;    // image column of Rt[.][0]
    const T* YL = (const T*)a.YL;
    const T* YR = (const T*)a.YR;
    for (int k = threadIdx.x; k < kLW * kLW; k += kT * kT) {
        const int r = k / kLW, q = k - r * kLW;
        const int gi = clampi_s(ti0 - kW + r, 0, a.rows - 1), gj = clampi_s(tj0 - kW + q, 0, a.cols - 1);
        L[r][q] = sld(YL, (size_t)gi * a.cols + gj);
    }
    for (int k = threadIdx.x; k < kLW * rw; k += kT * kT) {
        const int r = k / rw, q = k - r * rw;
        const int gi = clampi_s(ti0 - kW + r, 0, a.rows - 1), gj = clampi_s(rbase + q, 0, a.cols - 1);
        Rt[r][q] = sld(YR, (size_t)gi * a.cols + gj);
    }
    __syncthreads();
    const int li = threadIdx.x / kT, lj = threadIdx.x - li * kT;
    const int i = ti0 + li, j = tj0 + lj;
    if (i >= a.rows || j >= a.cols) return;

    // block matching, sums over window rows then columns as float32
    float best = __builtin_inff();
    int dbest = 0;
    for (int d = 0; d <= D; ++d) {
        float s = 0.0f;
        for (int aa = -kW; aa <= kW; ++aa) {
            const int r = li + kW + aa;
            for (int c = -kW; c <= kW; ++c) {
                const int gl = clampi_s(j + c, 0, a.cols - 1);
                const int gr = clampi_s(j + c - d, 0, a.cols - 1);
                s += fabsf(Rt[r][gr - rbase] - L[r][gl - (tj0 - kW)]);
            }
        }
        if (s < best) {
            best = s;
            dbest = d;
        }
    }

    // Gauss-Newton refinement: d <- d + sum(g r) / (sum(g^2) + eps), in [0, D + 1]
    float d = (float)dbest, A = 0.0f, E = 0.0f;
    for (int it = 0; it <= a.iters; ++it) {
        float sA = 0.0f, sB = 0.0f, sE = 0.0f;
        for (int aa = -kW; aa <= kW; ++aa) {
            const int r = li + kW + aa;
            for (int c = -kW; c <= kW; ++c) {
                const float xs = fminf(fmaxf((float)(j + c) - d, 0.0f), (float)(a.cols - 1));
                const int j0 = min((int)xs, a.cols - 1), j1 = min(j0 + 1, a.cols - 1);
                const float t = xs - (float)j0;
                const float r0 = Rt[r][j0 - rbase], r1 = Rt[r][j1 - rbase];
                const float g = r1 - r0;
                const float res = fmaf(t, g, r0) - L[r][clampi_s(j + c, 0, a.cols - 1) - (tj0 - kW)];
                sA = fmaf(g, g, sA);
                sB = fmaf(g, res, sB);
                sE += fabsf(res);
            }
        }
        A = sA;
        E = sE * (1.0f / 25.0f);
        if (it == a.iters) break;
        d = fminf(fmaxf(d + sB / (sA + 1e-6f), 0.0f), (float)(D + 1));
    }
    const float x = ((float)j - a.cx) / a.fx, y = ((float)i - a.cy) / a.fy;
    const float kappa = a.fx * a.baseline * sqrtf(fmaf(x, x, fmaf(y, y, 1.0f)));
    const bool ok = A >= a.texture && E <= a.residual && (float)j - d >= 0.0f;
    sst((T*)a.rho, (size_t)i * a.cols + j, ok ? d / kappa : __int_as_float(0x7fc00000));
}

}  // namespace

hipError_t launch_stereo(int storage, const StereoArgs& a, hipStream_t s) {
    const int blocks = ((a.rows + kT - 1) / kT) * ((a.cols + kT - 1) / kT);
    if (blocks == 0) return hipSuccess;
    if (a.dmax < 0 || a.dmax > kMaxD) return hipErrorInvalidValue;
    if (storage == SF_FP16)
        hipLaunchKernelGGL(k_stereo<__half>, dim3(blocks), dim3(kT * kT), 0, s, a);
    else
        hipLaunchKernelGGL(k_stereo<float>, dim3(blocks), dim3(kT * kT), 0, s, a);
    return hipGetLastError();
}

}  // namespace sflow
