// The learned update's network, all four layers over one output tile of one image, as a
// device function shared by the inference kernels (sflow_cnn.hip: k_net; sflow_kernels.hip:
// the filter's network-and-choice kernel).  Included by both; everything here is inline.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sflow {
namespace nettile {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t v) {
    return __builtin_bit_cast(float, (uint32_t)v << 16);
}
__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even (v_cvt_pk_bf16_f32)
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));
// two values rounded to BF16 (nearest even) in one instruction, a in the low half
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((fl2){a, b}, bf2));
}
// four BF16 values packed little-endian in two dwords, as the MFMA operand (element k = bits
// 16 k .. 16 k + 15): the same registers, no instruction
__device__ __forceinline__ s4 unpack4(uint2 v) { return __builtin_bit_cast(s4, v); }

// The four layers (inference: no layer input is kept) on one tile.  A block of 12 waves
// computes a kNetTH x kNetTW tile of one image's output (two blocks fit a CU's LDS).  It
// stages the input over the tile plus a 4-pixel margin (zero outside the image) in LDS; layer l = 0..3 then computes its
// output over the tile plus a (3 - l)-pixel margin from the other LDS buffer, setting the
// values outside the image to 0 (the zero padding the next layer reads); the last layer's three
// FP32 channels leave through LDS.  Each 16-pixel output row segment takes the nine MFMAs of
// k_conv in the same tap order with the operands' roles exchanged (weights as A, activations
// as B: D is the transposed product, each element the same sum of the same exact BF16
// products), then the same bias, ReLU and rounding, so the result is bitwise that of the four
// k_conv launches.  With the exchanged roles a lane receives four consecutive channels of one
// pixel and stores them with one 8-byte LDS write.
// Waves: wave w takes the 16 output columns 16 (w % 3) .. + 15 of a layer's region (3 x 16 =
// 48 >= its width) and a quarter of its rows, two rows at a time (two independent MFMA
// chains), sliding down them with the B operands of the input rows they read held in
// registers, so each input row is read from LDS once per wave.
constexpr int kNetTH = 16, kNetTW = 42;        // output tile
constexpr int kNetSegs = 3;                    // 16-pixel segments per region row (48 >= TW + 6)
constexpr int kNetWaves = kNetSegs * 4;        // a segment and a quarter of the rows each
constexpr int kNetThreads = 64 * kNetWaves;
constexpr int kNetPitch = 50;                  // LDS row pitch in pixels: TW + 8, and 32 + 15 + 2 < it
constexpr int kNetRowsX = kNetTH + 8;          // buffer X: the input (24 rows), layer 1's output (20)
constexpr int kNetRowsY = kNetTH + 6;          // buffer Y: layer 0's output (22), layer 2's output (18)
constexpr size_t kNetLds = (size_t)(kNetRowsX + kNetRowsY) * kNetPitch * 32;   // 73 600 bytes: two blocks per CU
static_assert(kNetTW + 8 == kNetPitch && 16 * (kNetSegs - 1) + 15 + 2 < kNetPitch &&
              kNetTW + 6 <= 16 * kNetSegs, "the segments cover every layer's region width");
static_assert(3 * kNetTH * kNetTW * 4 <= kNetRowsX * kNetPitch * 32, "output staging fits in X");

constexpr int kNetLayers = 4;

// LDS slot of channel quad q (8 bytes) of the pixel in column c of an activation row.  A
// B-operand read or an output write touches one quad of 16 consecutive pixels (32 bytes
// apart), which would put them on 8 of the 32 four-byte banks (4-way conflicts); XOR-ing the
// quad with bits 2-3 of the column gives the four pixels of equal column mod 4 four different
// slots, so any 16 consecutive pixels cover every bank once.
__device__ __forceinline__ int qslot(int c, int q) { return q ^ ((c >> 2) & 3); }

// The tile of the image whose pixels start at in + 16 base (BF16 NHWC 16, rows x cols) with
// its top-left output pixel at (ty0, tx0); w: BF16 [4][9][16 out][16 in], bias: FP32 [4][16].
// Leaves the three FP32 output channels of the tile in LDS at lds, as [3][kNetTH][kNetTW], and
// returns after a barrier (every thread of the block calls it).
__device__ __forceinline__ void net_tile(const uint16_t* in, const uint16_t* wts,
                                         const float* biases, int base, int rows, int cols,
                                         int ty0, int tx0, uint2* lds) {
    uint2* const X = lds;                                      // [row][pixel][channel quad]
    uint2* const Y = lds + (size_t)kNetRowsX * kNetPitch * 4;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15;           // A row: output channel; B column, D column: pixel
    const int quad = lane >> 4;          // A/B k block: input channels 4 quad .. +3; D rows:
                                         // output channels 4 quad .. +3
    {   // the input over the tile and a 4-pixel margin: 16-byte chunks, every load in flight
        // together (addresses outside the image read the first pixel and are zeroed)
        constexpr int NQ = kNetRowsX * kNetPitch * 2, NL = (NQ + kNetThreads - 1) / kNetThreads;
        uint4 vv[NL];
        bool inb[NL];
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int q = threadIdx.x + kNetThreads * m;
            const int px = q >> 1, half = q & 1;
            const int yy = ty0 - 4 + px / kNetPitch, xx = tx0 - 4 + px % kNetPitch;
            inb[m] = q < NQ && yy >= 0 && yy < rows && xx >= 0 && xx < cols;
            const size_t off = inb[m] ? ((size_t)base + (size_t)yy * cols + xx) * 16 + half * 8 : 0;
            vv[m] = *(const uint4*)(in + off);
        }
        // quads 2 half, 2 half + 1 of a pixel go to slots qslot(): the 16-byte chunk moves to
        // position half ^ (s >> 1) of the pixel, its 8-byte halves swapped when s is odd
        uint4* X4 = reinterpret_cast<uint4*>(X);
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int q = threadIdx.x + kNetThreads * m;
            const int sw = ((q >> 1) % kNetPitch >> 2) & 3;
            uint4 v = inb[m] ? vv[m] : make_uint4(0u, 0u, 0u, 0u);
            if (sw & 1) v = make_uint4(v.z, v.w, v.x, v.y);
            if (q < NQ) X4[q ^ (sw >> 1)] = v;
        }
    }
    float* const out32 = reinterpret_cast<float*>(X);         // [3][TH][TW], after layer 2
    const int x0 = 16 * (wave % kNetSegs);
    const int px = x0 + col;                                  // this lane's output pixel column
    for (int l = 0; l < kNetLayers; ++l) {
        const uint2* src = (l & 1) ? Y : X;
        uint2* dst = (l & 1) ? X : Y;
        const int halo = 3 - l;                                // margin of this layer's output
        const int R = kNetTH + 2 * halo, W = kNetTW + 2 * halo;
        const int rq = wave / kNetSegs;
        const int r0 = rq * R / 4, r1 = (rq + 1) * R / 4;
        s4 wv[9];
#pragma unroll
        for (int tp = 0; tp < 9; ++tp)
            wv[tp] = unpack4(*(const uint2*)(wts + (((size_t)l * 9 + tp) * 16 + col) * 16 + 4 * quad));
        float bias[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) bias[k] = biases[l * 16 + 4 * quad + k];
        const int gx = tx0 - halo + px;
        const bool col_in = px < W && gx >= 0 && gx < cols;
        __syncthreads();   // the previous layer's output (or the staged input) is complete
        auto load_row = [&](s4 (&g)[3], int row) {
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
                g[dx] = unpack4(src[((size_t)row * kNetPitch + x0 + col + dx) * 4 +
                                    qslot(x0 + col + dx, quad)]);
        };
        // output row r: D[4 quad + k][col] is channel 4 quad + k of pixel px
        auto store_row = [&](int r, const f4& acc) {
            if (l < kNetLayers - 1) {
                const int gy = ty0 - halo + r;
                const bool in = col_in && gy >= 0 && gy < rows;
                const uint32_t lo = f2bf2(fmaxf(acc[0] + bias[0], 0.0f), fmaxf(acc[1] + bias[1], 0.0f));
                const uint32_t hi = f2bf2(fmaxf(acc[2] + bias[2], 0.0f), fmaxf(acc[3] + bias[3], 0.0f));
                dst[((size_t)r * kNetPitch + px) * 4 + qslot(px, quad)] =
                    make_uint2(in ? lo : 0u, in ? hi : 0u);
            } else if (quad == 0 && px < kNetTW) {
#pragma unroll
                for (int k = 0; k < 3; ++k) out32[(k * kNetTH + r) * kNetTW + px] = acc[k] + bias[k];
            }
        };
        // B operands of the input rows r .. r + 3 (output rows r, r + 1 read r .. r + 2 and
        // r + 1 .. r + 3), columns x0 + col + 0..2
        s4 f[4][3];
        if (r0 < r1) {
            load_row(f[0], r0);
            load_row(f[1], r0 + 1);
        }
        int r = r0;
        for (; r + 1 < r1; r += 2) {
            load_row(f[2], r + 2);
            load_row(f[3], r + 3);
            f4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wv[dy * 3 + dx], f[dy][dx], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wv[dy * 3 + dx], f[dy + 1][dx], acc1, 0, 0, 0);
                }
            store_row(r, acc0);
            store_row(r + 1, acc1);
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                f[0][dx] = f[2][dx];
                f[1][dx] = f[3][dx];
            }
        }
        if (r < r1) {   // an odd row left
            load_row(f[2], r + 2);
            f4 acc0 = {0, 0, 0, 0};
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
                    acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wv[dy * 3 + dx], f[dy][dx], acc0, 0, 0, 0);
            store_row(r, acc0);
        }
    }
    __syncthreads();
}

}  // namespace nettile
}  // namespace sflow
