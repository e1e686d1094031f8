// The learned update's network on gfx950: a 4-layer 3x3 convolutional network
// (9 -> 16 -> 16 -> 16 -> 3 channels, ReLU after the first three layers, zero padding) in
// BF16 on the matrix cores with FP32 accumulation, and the kernels that train it.
//
// Activations are NHWC with 16 BF16 channels per pixel (32 bytes; unused channels are 0),
// for a list of images stored one after the other ("segments"), each image's pixel range
// padded to a multiple of 16 so that a wave's 16 pixels never straddle two images.
//
// Convolution as an implicit GEMM: a wave computes 16 pixels x 16 output channels with nine
// v_mfma_f32_16x16x16_bf16 (one per tap, K = 16 input channels), its A operands read from an
// LDS copy of the block's input patch.  Operand layout of
// that instruction (64 lanes): lane l holds A[l%16][4(l/16) .. +3] and B[4(l/16) .. +3][l%16]
// and receives D[4(l/16) .. +3][l%16].  Here A[i][k] = input channel k of pixel i shifted by
// the tap, B[k][j] = weight (tap, k -> j), D[i][j] = output channel j of pixel i.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "sflow_cnn.h"
#include "sflow_net_tile.h"

namespace sflow {
namespace {

using nettile::s4;
using nettile::f4;
using nettile::bf2f;
using nettile::f2bf;
using nettile::unpack4;

// the image a 16-pixel group belongs to
__device__ __forceinline__ int find_seg(const CnnSegs& s, int p) {
    int k = 0;
    while (k + 1 < s.n && s.base[k + 1] <= p) ++k;
    return k;
}

// 3x3 convolution layer over all images.  A block of 4 waves computes a 16 x 16 pixel tile:
// it stages the tile's 18 x 18 input patch (16 BF16 channels per pixel, zero outside the image,
// optionally masked) in LDS, and each wave computes 4 rows of 16 pixels x 16 output channels,
// nine MFMAs per row (one per tap) with the weights held in registers.
constexpr int kConvTile = 16, kConvPatch = kConvTile + 2;

template <bool OUT_F32>
__global__ void __launch_bounds__(256) k_conv(ConvArgs a) {
    __shared__ uint2 patch[kConvPatch * kConvPatch * 4];   // [y][x][channel quad]
    const int b = blockIdx.x;
    int sgi = 0;
    while (sgi + 1 < a.segs.n && a.tblk[sgi + 1] <= b) ++sgi;
    const int base = a.segs.base[sgi], rows = a.segs.rows[sgi], cols = a.segs.cols[sgi];
    const int t = b - a.tblk[sgi];
    const int tiles_x = (cols + kConvTile - 1) / kConvTile;
    const int ty0 = (t / tiles_x) * kConvTile, tx0 = (t % tiles_x) * kConvTile;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15;           // A row: pixel column within the tile; D column: channel
    const int quad = lane >> 4;          // A/B k block: input channels 4 quad .. +3
    // B: weight[tap][out j = lane % 16][in 4 (lane / 16) .. +3], loaded first so that its
    // latency overlaps the patch loads'
    s4 bv[9];
#pragma unroll
    for (int tp = 0; tp < 9; ++tp)
        bv[tp] = unpack4(*(const uint2*)(a.w + ((size_t)tp * 16 + col) * 16 + 4 * quad));
    const float bias = a.bias ? a.bias[col] : 0.0f;
    {   // every load of the patch in flight together (addresses outside the image read the
        // first pixel and are zeroed), then the LDS stores
        constexpr int NQ = kConvPatch * kConvPatch * 4, NL = (NQ + 255) / 256;
        uint2 vv[NL], mm[NL];
        bool inb[NL];
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int q = threadIdx.x + 256 * m;
            const int px = q >> 2, quad = q & 3;
            const int yy = ty0 - 1 + px / kConvPatch, xx = tx0 - 1 + px % kConvPatch;
            inb[m] = q < NQ && yy >= 0 && yy < rows && xx >= 0 && xx < cols;
            const size_t off = inb[m] ? ((size_t)base + (size_t)yy * cols + xx) * 16 + quad * 4 : 0;
            vv[m] = *(const uint2*)(a.in + off);
            if (a.mask) mm[m] = *(const uint2*)(a.mask + off);
        }
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int q = threadIdx.x + 256 * m;
            if (q >= NQ) continue;
            uint2 v = inb[m] ? vv[m] : make_uint2(0u, 0u);
            if (a.mask) {
                const uint2 mk = mm[m];
                if (bf2f((uint16_t)(mk.x & 0xffff)) <= 0.0f) v.x &= 0xffff0000u;
                if (bf2f((uint16_t)(mk.x >> 16)) <= 0.0f) v.x &= 0x0000ffffu;
                if (bf2f((uint16_t)(mk.y & 0xffff)) <= 0.0f) v.y &= 0xffff0000u;
                if (bf2f((uint16_t)(mk.y >> 16)) <= 0.0f) v.y &= 0x0000ffffu;
            }
            patch[q] = v;
        }
    }
    __syncthreads();
    // results go to an LDS copy of the output tile first, then every thread writes one pixel
    // whole (two 16-byte stores, or three channel planes), instead of 2-byte stores per lane
    __shared__ uint4 tile16[kConvTile * kConvTile * 2];   // BF16 [pixel][16 channels]
    __shared__ float tile32[3][kConvTile * kConvTile];    // FP32 [channel][pixel]
    uint16_t* t16 = reinterpret_cast<uint16_t*>(tile16);
#pragma unroll
    for (int rr = 0; rr < kConvTile / 4; ++rr) {
        const int row = wave * (kConvTile / 4) + rr;     // tile row of this wave
        f4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) {
            const int dy = tp / 3 - 1, dx = tp % 3 - 1;
            const s4 av = unpack4(patch[((row + 1 + dy) * kConvPatch + (col + 1 + dx)) * 4 + quad]);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv[tp], acc, 0, 0, 0);
        }
        // D[4 (lane / 16) + r][lane % 16]: pixel column 4 quad + r of this row, channel col
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int px = row * kConvTile + 4 * quad + r;
            float v = acc[r] + bias;
            if (a.relu) v = fmaxf(v, 0.0f);
            if (OUT_F32) {
                if (col < 3) tile32[col][px] = v;
            } else {
                t16[px * 16 + col] = col < a.nout ? f2bf(v) : (uint16_t)0;
            }
        }
    }
    __syncthreads();
    const int px = threadIdx.x;                           // one pixel of the tile per thread
    const int y = ty0 + px / kConvTile, x = tx0 + px % kConvTile;
    if (y >= rows || x >= cols) return;
    const size_t i = (size_t)base + (size_t)y * cols + x;
    if (OUT_F32) {
        for (int c = 0; c < a.nout && c < 3; ++c) a.out_f32[(size_t)c * a.segs.total + i] = tile32[c][px];
    } else {
        uint4* o = reinterpret_cast<uint4*>(a.out + i * 16);
        o[0] = tile16[px * 2];
        o[1] = tile16[px * 2 + 1];
    }
}

// The four layers in one launch (inference): one block per 16 x 42 output tile of one image
// (nettile::net_tile), bitwise the four k_conv launches.
__global__ void __launch_bounds__(nettile::kNetThreads) k_net(NetArgs a) {
    extern __shared__ uint2 net_lds[];
    const int b = blockIdx.x;
    int sgi = 0;
    while (sgi + 1 < a.segs.n && a.tblk[sgi + 1] <= b) ++sgi;
    const int base = a.segs.base[sgi], rows = a.segs.rows[sgi], cols = a.segs.cols[sgi];
    const int t = b - a.tblk[sgi];
    using namespace nettile;
    const int tiles_x = (cols + kNetTW - 1) / kNetTW;
    const int ty0 = (t / tiles_x) * kNetTH, tx0 = (t % tiles_x) * kNetTW;
    net_tile(a.in, a.w, a.bias, base, rows, cols, ty0, tx0, net_lds);
    const float* out32 = reinterpret_cast<const float*>(net_lds);
    for (int p = threadIdx.x; p < kNetTH * kNetTW; p += kNetThreads) {
        const int y = ty0 + p / kNetTW, x = tx0 + p % kNetTW;
        if (y >= rows || x >= cols) continue;
        const size_t i = (size_t)base + (size_t)y * cols + x;
#pragma unroll
        for (int c = 0; c < 3; ++c) a.out_f32[(size_t)c * a.segs.total + i] = out32[c * kNetTH * kNetTW + p];
    }
}

// Weight and bias gradients of one layer: dW[t][c][n] = sum_p in[p + t][c] g[p][n],
// db[n] = sum_p g[p][n], with g = dout masked by (act > 0) when act is given.  Each wave
// reduces `per_wave` 16-pixel groups on the matrix cores and adds its partial sums to the
// FP32 gradient (A = input channels x pixels, B = pixels x output channels).
__global__ void __launch_bounds__(256) k_conv_dw(DwArgs a) {
    const int lane = threadIdx.x & 63;
    const int wv = (blockIdx.x * 256 + threadIdx.x) >> 6;
    const int g0 = wv * a.per_wave;
    const int ngroups = a.segs.total / 16;
    if (g0 >= ngroups) return;
    const int g1 = min(g0 + a.per_wave, ngroups);
    f4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = (f4){0, 0, 0, 0};
    float dbs = 0.0f;
    const int cA = lane & 15;          // A row: input channel
    const int k0 = 4 * (lane >> 4);    // A/B k: pixel offset within the group
    for (int g = g0; g < g1; ++g) {
        const int p0 = g * 16;
        const int sgi = find_seg(a.segs, p0);
        const int base = a.segs.base[sgi], rows = a.segs.rows[sgi], cols = a.segs.cols[sgi];
        const int npx = rows * cols;
        // B: g[p][n] for the lane's 4 pixels, n = lane%16
        s4 bv;
        int py[4], px[4];
        bool pv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = p0 - base + k0 + r;
            pv[r] = i < npx;
            py[r] = pv[r] ? i / cols : 0;
            px[r] = pv[r] ? i - py[r] * cols : 0;
            uint16_t gv = 0;
            if (pv[r]) {
                const size_t off = ((size_t)base + i) * 16 + cA;
                gv = a.dout[off];
                if (a.act && bf2f(a.act[off]) <= 0.0f) gv = 0;
            }
            bv[r] = (short)gv;
            dbs += bf2f(gv);
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            s4 av;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int yy = py[r] + dy, xx = px[r] + dx;
                uint16_t v = 0;
                if (pv[r] && yy >= 0 && yy < rows && xx >= 0 && xx < cols)
                    v = a.in[((size_t)base + (size_t)yy * cols + xx) * 16 + cA];
                av[r] = (short)v;
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[t], 0, 0, 0);
        }
    }
    // D[i = c][j = n]: lane holds c = 4(lane/16) + r, n = lane%16
    const int n = lane & 15;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 4 * (lane >> 4) + r;
            atomicAdd(&a.dw[(t * 16 + c) * 16 + n], acc[t][r]);
        }
    // bias: lanes sharing n = lane%16 hold disjoint pixel sets; the B values of channel n are
    // those with cA == n, i.e. lanes whose lane%16 == n
    atomicAdd(&a.db[lane & 15], dbs);
}

// loss: Charbonnier endpoint error between the network's output (FP32 planes, 3 channels) and
// the target; writes d loss / d output as BF16 NHWC (16 channels, 3 used; one pixel's 32 bytes
// in two 16-byte stores) and adds the loss: a wave sum by lane shuffles, a block sum through
// LDS, one atomic add per block.
__global__ void __launch_bounds__(256) k_loss(LossArgs a) {
    __shared__ float wsum[256 / 64];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool in = p < a.segs.total;
    float d[3] = {0, 0, 0};
    float n = 1.0f, l = 0.0f;
    bool valid = false;
    if (in) {
        const int sgi = find_seg(a.segs, p);
        const int i = p - a.segs.base[sgi];
        valid = i < a.segs.rows[sgi] * a.segs.cols[sgi];
        if (valid) {
            float s2 = a.eps * a.eps;
            for (int c = 0; c < 3; ++c) {
                d[c] = a.out[(size_t)c * a.segs.total + p] - a.target[(size_t)c * a.segs.total + p];
                s2 = fmaf(d[c], d[c], s2);
            }
            n = sqrtf(s2);
            l = n * a.inv_count;
        }
        uint32_t g[3];
        for (int c = 0; c < 3; ++c) g[c] = valid ? f2bf(d[c] / n * a.inv_count) : 0u;
        uint4* o = reinterpret_cast<uint4*>(a.dout + (size_t)p * 16);
        o[0] = make_uint4(g[0] | (g[1] << 16), g[2], 0u, 0u);
        o[1] = make_uint4(0u, 0u, 0u, 0u);
    }
    // every lane of the block takes part in the sums (lanes past the end add 0)
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wsum[wave] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int w = 0; w < 256 / 64; ++w) t += wsum[w];
        atomicAdd(a.loss, t);
    }
}

// FP32 planar inputs (C planes of `total` pixels) -> BF16 NHWC 16 channels
__global__ void __launch_bounds__(256) k_pack_inputs(const float* in, int C, int total,
                                                     uint16_t* out) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= total) return;
    for (int c = 0; c < 16; ++c)
        out[(size_t)p * 16 + c] = c < C ? f2bf(in[(size_t)c * total + p]) : (uint16_t)0;
}

// Adam on the FP32 master parameters, then the BF16 weights of the forward kernel
// ([tap][out 16][in 16]) and of the input-gradient kernel (taps mirrored, in/out swapped).
__global__ void __launch_bounds__(256) k_adam(AdamArgs a) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q < a.nparams && a.lr > 0.0f) {
        const float g = a.grad[q];
        const float m = a.b1 * a.m[q] + (1.0f - a.b1) * g;
        const float v = a.b2 * a.v[q] + (1.0f - a.b2) * g * g;
        a.m[q] = m;
        a.v[q] = v;
        a.params[q] -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
    }
}

__global__ void __launch_bounds__(256) k_pack_weights(PackArgs a) {
    const int q = blockIdx.x * 256 + threadIdx.x;     // one entry of the packed 4 x 9 x 16 x 16
    if (q >= 4 * 9 * 256) return;
    const int l = q / (9 * 256);
    const int rem = q - l * 9 * 256;
    const int t = rem / 256;
    const int n = (rem / 16) % 16;   // output channel of the forward kernel
    const int c = rem % 16;          // input channel
    const int cin = a.cin[l], cout = a.cout[l];
    const float* W = a.params + a.woff[l];             // (3, 3, cin, cout) row-major
    const float vf = (c < cin && n < cout) ? W[(t * cin + c) * cout + n] : 0.0f;
    a.wf[q] = f2bf(vf);
    // input-gradient kernel of layer l: out channel = forward input c', in channel = forward
    // output n', tap mirrored: weight (8 - t, c' = n, n' = c)
    const float vb = (n < cin && c < cout) ? W[((8 - t) * cin + n) * cout + c] : 0.0f;
    a.wb[q] = f2bf(vb);
    if (t == 0 && c == 0) a.bias[l * 16 + n] = n < cout ? a.params[a.boff[l] + n] : 0.0f;
}

__global__ void __launch_bounds__(256) k_gather_grads(GradArgs a) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= kCnnParams) return;
    int l = 0;
    while (l + 1 < kCnnLayers && a.woff[l + 1] <= q) ++l;
    const int cin = a.cin[l], cout = a.cout[l];
    if (q < a.boff[l]) {
        const int idx = q - a.woff[l];
        const int t = idx / (cin * cout);
        const int c = (idx / cout) % cin;
        const int n = idx % cout;
        a.grad[q] = a.dw[((size_t)(l * 9 + t) * 16 + c) * 16 + n];
    } else {
        a.grad[q] = a.db[l * 16 + (q - a.boff[l])];
    }
}

__global__ void __launch_bounds__(256) k_planes_in(CnnSegs sg, const float* src, int C, float* dst) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= sg.total) return;
    const int k = find_seg(sg, p);
    const int i = p - sg.base[k];
    const int npx = sg.rows[k] * sg.cols[k];
    for (int c = 0; c < C; ++c)
        dst[(size_t)c * sg.total + p] = i < npx ? src[(size_t)sg.off[k] * C + (size_t)c * npx + i] : 0.0f;
}

__global__ void __launch_bounds__(256) k_planes_out(CnnSegs sg, const float* src, int C, float* dst) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= sg.total) return;
    const int k = find_seg(sg, p);
    const int i = p - sg.base[k];
    const int npx = sg.rows[k] * sg.cols[k];
    if (i >= npx) return;
    for (int c = 0; c < C; ++c)
        dst[(size_t)sg.off[k] * C + (size_t)c * npx + i] = src[(size_t)c * sg.total + p];
}

}  // namespace

hipError_t launch_gather_grads(const GradArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_grads, dim3((kCnnParams + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_planes_in(const CnnSegs& sg, const float* src, int C, float* dst, hipStream_t s) {
    const int blocks = (sg.total + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_planes_in, dim3(blocks), dim3(256), 0, s, sg, src, C, dst);
    return hipGetLastError();
}

hipError_t launch_planes_out(const CnnSegs& sg, const float* src, int C, float* dst, hipStream_t s) {
    const int blocks = (sg.total + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_planes_out, dim3(blocks), dim3(256), 0, s, sg, src, C, dst);
    return hipGetLastError();
}

hipError_t launch_conv(const ConvArgs& args, bool out_f32, hipStream_t s) {
    ConvArgs a = args;
    int blocks = 0;
    for (int k = 0; k < a.segs.n; ++k) {
        a.tblk[k] = blocks;
        blocks += ((a.segs.rows[k] + kConvTile - 1) / kConvTile) *
                  ((a.segs.cols[k] + kConvTile - 1) / kConvTile);
    }
    a.tblk[a.segs.n] = blocks;
    if (blocks == 0) return hipSuccess;
    if (out_f32)
        hipLaunchKernelGGL(k_conv<true>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_conv<false>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_net(const NetArgs& args, hipStream_t s) {
    static std::atomic<uint64_t> prepared{0};   // devices the LDS limit was raised on
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = 1ull << (dev & 63);
    if (!(prepared.load() & bit)) {
        e = hipFuncSetAttribute((const void*)k_net, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)nettile::kNetLds);
        if (e != hipSuccess) return e;
        prepared.fetch_or(bit);
    }
    NetArgs a = args;
    int blocks = 0;
    for (int k = 0; k < a.segs.n; ++k) {
        a.tblk[k] = blocks;
        blocks += ((a.segs.rows[k] + nettile::kNetTH - 1) / nettile::kNetTH) *
                  ((a.segs.cols[k] + nettile::kNetTW - 1) / nettile::kNetTW);
    }
    a.tblk[a.segs.n] = blocks;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_net, dim3(blocks), dim3(nettile::kNetThreads), nettile::kNetLds, s, a);
    return hipGetLastError();
}

hipError_t launch_conv_dw(const DwArgs& a, hipStream_t s) {
    const int groups = a.segs.total / 16;
    const int waves = (groups + a.per_wave - 1) / a.per_wave;
    const int blocks = (waves + 3) / 4;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_conv_dw, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_loss(const LossArgs& a, hipStream_t s) {
    const int blocks = (a.segs.total + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_loss, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pack_inputs(const float* in, int C, int total, uint16_t* out, hipStream_t s) {
    const int blocks = (total + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_inputs, dim3(blocks), dim3(256), 0, s, in, C, total, out);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((a.nparams + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pack_weights(const PackArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_weights, dim3((4 * 9 * 256 + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sflow
