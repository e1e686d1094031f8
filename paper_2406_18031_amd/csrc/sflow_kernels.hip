// gfx950 kernels of the structure-flow filter.
//
// k_step is the hot path: one workgroup owns one output tile of one pyramid level and runs,
// for that tile, every stage of the level's predictor-update block (Section "Filter
// Architecture") on the tile plus a halo held on chip:
//   prediction  N upwind column/row half-steps (Section "Numerical prediction"),
//   image model 5x5 Gaussian-weighted linear fit as separable passes (eq:img_model),
//   depth model occlusion-aware one-sided differences (eq:dominant_b1/b2),
//   update      the 3x3 least-squares system (eq:LS_update) solved in residual form
//               around the prior: x = x0 + alpha a_Y + beta a_rho (2x2 inner system),
//   smoothing   N_s passes of the 5x5 average,
//   rho update  eq:cost_invdepth.
// The halo is max(N, 2) + 2 N_s pixels per side: each half-step invalidates one pixel on
// each interior side of the region, each 5x5 pass two.  The region (at most 64 x 64) lives in
// registers: lane l of wave w holds column l of the wave's strip of rows, so column
// neighbours come from DPP lane shifts and row neighbours from the same lane's registers,
// with only the strip-boundary rows exchanged through LDS (one barrier per step).  Geometry
// (unit ray, tangent basis, pixel spacing) is recomputed from the pinhole intrinsics in
// registers instead of being read from memory.
#include <atomic>

#include "sflow_internal.h"
#include "sflow_net_tile.h"

namespace sflow {
namespace {

__device__ __forceinline__ float ldv(const float* p, size_t i) { return p[i]; }
__device__ __forceinline__ float ldv(const __half* p, size_t i) { return __half2float(p[i]); }
__device__ __forceinline__ void stv(float* p, size_t i, float v) { p[i] = v; }
__device__ __forceinline__ void stv(__half* p, size_t i, float v) { p[i] = __float2half(v); }

// The level table is written by the host before a launch and never by a kernel, so kernels
// read it through the constant address space: the compiler may then use scalar loads for it
// (uniform, cached, issued early) instead of vector loads ordered behind the kernel's stores.
typedef const __attribute__((address_space(4))) LevelDev ConstLevelDev;
__device__ __forceinline__ ConstLevelDev& level_entry(const LevelDev* tab, int e) {
    return ((ConstLevelDev*)tab)[e];
}
__device__ __forceinline__ int level_block0(const LevelDev* tab, int e) {
    return ((ConstLevelDev*)tab)[e].block0;
}

template <typename T> __device__ __forceinline__ float flow_in_scale(ConstLevelDev& L);
template <> __device__ __forceinline__ float flow_in_scale<float>(ConstLevelDev&) { return 1.0f; }
template <> __device__ __forceinline__ float flow_in_scale<__half>(ConstLevelDev& L) {
    return 1.0f / L.qscale;
}
template <typename T> __device__ __forceinline__ float flow_out_scale(ConstLevelDev& L);
template <> __device__ __forceinline__ float flow_out_scale<float>(ConstLevelDev&) { return 1.0f; }
template <> __device__ __forceinline__ float flow_out_scale<__half>(ConstLevelDev& L) {
    return L.qscale;
}

// 1-D Gaussian taps g = [1, 4, 6, 4, 1] / 16 (exact in binary)
__device__ __forceinline__ float gtap(int a) {
    return a == 0 ? 0.375f : ((a == 1 || a == -1) ? 0.25f : 0.0625f);
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Pinhole geometry of pixel (i, j).  With r = ((j - cx)/fx, (i - cy)/fy, 1) = (x, y, 1),
// eta = r/|r| and the next column's ray r_n = r +- e_x/fx (the previous column in the last
// column), P_eta eta_n is parallel to P_eta e_x, which gives in closed form
//   b1 = (e_x - eta eta_x)/sqrt(1 - eta_x^2),  b2 = eta x b1 = (0, eta_z, -eta_y)/sqrt(..),
//   dmu = sqrt(1 - eta_x^2)/(fx |r_n|),
// and for any w the column/row optical flow and normal component
//   u = b1.w/dmu = fx|r_n| (w_x - x (y w_y + w_z)/(1 + y^2)),
//   v = b2.w/dmu = fx|r_n| |r| (w_y - y w_z)/(1 + y^2),
//   s = <eta, w> = (x w_x + y w_y + w_z)/|r|.
struct Geo {
    float x, y, rinv, r, fxrn, inv1py2;
};

__device__ __forceinline__ Geo pixel_geo(ConstLevelDev& L, int i, int j) {
    Geo g;
    g.x = fmaf((float)j, L.ifx, -L.cxn);
    g.y = fmaf((float)i, L.ify, -L.cyn);
    const float yy1 = fmaf(g.y, g.y, 1.0f);
    const float r2 = fmaf(g.x, g.x, yy1);
    g.rinv = rsqrtf(r2);
    g.r = r2 * g.rinv;
    const float xn = g.x + (j < L.cols - 1 ? L.ifx : -L.ifx);
    g.fxrn = L.fx * sqrtf(fmaf(xn, xn, yy1));
    g.inv1py2 = 1.0f / yy1;
    return g;
}

// dmu = sqrt(1 - eta_x^2) / (fx |r_n|), computed as in the update stage of k_step; on a general
// grid 1 / |b1/dmu| from the level's geometry table, as there
__device__ __forceinline__ float pixel_dmu(ConstLevelDev& L, int i, int j) {
    if (L.geo) {
        const size_t plane = (size_t)L.rows * L.gpitch, o = (size_t)i * L.gpitch + j;
        const float a = L.geo[o], b = L.geo[plane + o], c = L.geo[2 * plane + o];
        return rsqrtf(fmaf(a, a, fmaf(b, b, c * c)));
    }
    const float x = fmaf((float)j, L.ifx, -L.cxn);
    const float xn = x + (j < L.cols - 1 ? L.ifx : -L.ifx);
    const float y = fmaf((float)i, L.ify, -L.cyn);
    const float yy1 = fmaf(y, y, 1.0f);
    const float r2 = fmaf(x, x, yy1);
    const float rinv = rsqrtf(r2);
    const float fxrn = L.fx * __builtin_amdgcn_sqrtf(fmaf(xn, xn, yy1));
    const float q = __builtin_amdgcn_sqrtf(fmaf(y, y, 1.0f)) * rinv;
    return q * __builtin_amdgcn_rcpf(fxrn);
}

__device__ __forceinline__ float flow_u(const Geo& g, float wx, float wy, float wz) {
    return g.fxrn * (wx - g.x * fmaf(g.y, wy, wz) * g.inv1py2);
}
__device__ __forceinline__ float flow_v(const Geo& g, float wx, float wy, float wz) {
    (void)wx;
    return g.fxrn * g.r * (wy - g.y * wz) * g.inv1py2;
}
__device__ __forceinline__ float normal_s(const Geo& g, float wx, float wy, float wz) {
    return fmaf(g.x, wx, fmaf(g.y, wy, wz)) * g.rinv;
}

// one-sided difference of smaller magnitude, forward on a tie; NaN-aware (missing depth)
__device__ __forceinline__ float minabs_diff(float c, float nxt, float prv) {
    const float dp = nxt - c;
    const float dm = c - prv;
    const bool np = isnan(dp), nm = isnan(dm);
    if (np && nm) return 0.0f;
    if (np) return dm;
    if (nm) return dp;
    return fabsf(dp) <= fabsf(dm) ? dp : dm;
}

// ------------------------------------------------------------------------------------------
// fused level step
// ------------------------------------------------------------------------------------------
// Lane l of wave w holds column gj0 + l of region rows [w R, w R + R) in registers, R = kRPW.
// Cross-lane moves must run with every lane of the wave active (a DPP read from a lane that
// EXEC disables does not return that lane's value), so they are only ever called as plain
// statements, never inside a conditional expression or a lane-dependent branch.  Lanes whose
// source lies outside the wave read 0; those are region-edge lanes, never valid output.
__device__ __forceinline__ float dpp_prev(float v) {   // value of the lane to the left
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(
        __builtin_bit_cast(int, v), 0x138 /* wave_shr:1 */, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_next(float v) {   // value of the lane to the right
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(
        __builtin_bit_cast(int, v), 0x130 /* wave_shl:1 */, 0xF, 0xF, true));
}

// acc[k] -= f[k] of the lane to the right * c, for every k, as v_fmac_f32 with the lane shift
// on its first source (the compiler folds lane shifts into multiplies and adds but not into
// fmac).  The compiler does not account for the wait states a shifted read needs after the
// instruction that wrote its source (2 after a VALU write, 5 after an EXEC write), so the
// block starts with 5 of its own; the reads inside the block are of registers written before
// it.  Same rules as dpp_next: every lane active; lanes past the wave's end read 0.
template <int NF>
__device__ __forceinline__ void fmac_next_neg(float (&acc)[NF], const float (&f)[NF], float c) {
    static_assert(NF == 4 || NF == 8, "four or eight fields");
    if constexpr (NF == 4) {
        asm("s_nop 4\n\t"
            "v_fmac_f32_dpp %0, %4, -%8 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
            "v_fmac_f32_dpp %1, %5, -%8 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
            "v_fmac_f32_dpp %2, %6, -%8 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
            "v_fmac_f32_dpp %3, %7, -%8 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
            : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3])
            : "v"(f[0]), "v"(f[1]), "v"(f[2]), "v"(f[3]), "v"(c));
    } else {
        asm("s_nop 4\n\t"
            "v_fmac_f32_dpp %0, %8, -%16 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
            "v_fmac_f32_dpp %1, %9, -%16 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
            "v_fmac_f32_dpp %2, %10, -%16 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
            "v_fmac_f32_dpp %3, %11, -%16 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
            "v_fmac_f32_dpp %4, %12, -%16 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
            "v_fmac_f32_dpp %5, %13, -%16 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
            "v_fmac_f32_dpp %6, %14, -%16 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
            "v_fmac_f32_dpp %7, %15, -%16 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
            : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]),
              "+v"(acc[4]), "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7])
            : "v"(f[0]), "v"(f[1]), "v"(f[2]), "v"(f[3]),
              "v"(f[4]), "v"(f[5]), "v"(f[6]), "v"(f[7]), "v"(c));
    }
}

// Column neighbours with clamping at the image's left/right border (the border pixel is its
// own neighbour).  BORDER is false for tiles that touch neither border.
template <bool BORDER>
__device__ __forceinline__ float nb_prev(float v, bool at_left) {
    const float p = dpp_prev(v);
    return BORDER && at_left ? v : p;
}
template <bool BORDER>
__device__ __forceinline__ float nb_next(float v, bool at_right) {
    const float p = dpp_next(v);
    return BORDER && at_right ? v : p;
}
__device__ __forceinline__ float clamp_prev(float v, bool keep) {
    const float p = dpp_prev(v);
    return keep ? v : p;
}
__device__ __forceinline__ float clamp_next(float v, bool keep) {
    const float p = dpp_next(v);
    return keep ? v : p;
}

// Geometry of pixel (i, j) for the register-strip kernel: y, 1/|r|, fx |r_n|, x/(1 + y^2)
// and B = fx |r_n| |r| / (1 + y^2) (see pixel_geo for the closed forms).
__device__ __forceinline__ void row_geo(ConstLevelDev& L, int i, float x, float xn, float& y,
                                        float& rinv, float& fxrn, float& xi, float& B) {
    y = fmaf((float)i, L.ify, -L.cyn);
    const float yy1 = fmaf(y, y, 1.0f);
    const float r2 = fmaf(x, x, yy1);
    rinv = rsqrtf(r2);
    fxrn = L.fx * __builtin_amdgcn_sqrtf(fmaf(xn, xn, yy1));
    const float inv = __builtin_amdgcn_rcpf(yy1);   // 1 ulp reciprocal
    xi = x * inv;
    B = fxrn * (r2 * rinv) * inv;
}

// Largest magnitude a stored flow value may have: beyond it (or NaN) the store is flagged.
template <typename T> __device__ __forceinline__ float stored_max();
template <> __device__ __forceinline__ float stored_max<float>() { return 3.4028234663852886e38f; }
template <> __device__ __forceinline__ float stored_max<__half>() { return 65504.0f; }

// Sets the stream's bit of the watchdog word if any lane of the wave stored a flagged value:
// one atomic from the wave's first flagged lane (called by every lane of the wave).
__device__ __forceinline__ void flag_nonfinite(bool bad, int lane, ConstLevelDev& L) {
    const unsigned long long m = __ballot(bad);
    if (m != 0ull && lane == __ffsll((long long)m) - 1)
        atomicOr(L.numeric, 1ull << L.stream);
}

constexpr int kNW = kBlock / 64;        // waves per block
constexpr int kRPW = kRegion / kNW;     // region rows per wave

// Geometry of the pixels a lane holds in the fused level kernel (its column, the wave's kRPW
// rows and the rows just above and below the strip), giving for a flow w the column and row
// optical flow u = b1.w / dmu, v = b2.w / dmu (eq:oflow_numeric), the normal component
// s = <eta, w>, and for the update the frame (eta, b1, b2, dmu).
//
// Pinhole grid: closed forms from the intrinsics (see pixel_geo), nothing read from memory.
struct PinholeRows {
    static constexpr bool kB2xZero = true;   // b2 has no x component
    float x, xn;
    float y[kRPW], rinv[kRPW], fxrn[kRPW], xi[kRPW], B[kRPW];
    float yA, BA, yBl, BBl;   // rows just above / below the strip (y and B)
    __device__ __forceinline__ void load(ConstLevelDev& L, int wi0, int j) {
        x = fmaf((float)j, L.ifx, -L.cxn);
        xn = x + (j < L.cols - 1 ? L.ifx : -L.ifx);
#pragma unroll
        for (int r = 0; r < kRPW; ++r) row_geo(L, wi0 + r, x, xn, y[r], rinv[r], fxrn[r], xi[r], B[r]);
        // same arithmetic as the owning wave, so results do not depend on where strips start
        float t0, t1, t2;
        row_geo(L, wi0 - 1, x, xn, yA, t0, t1, t2, BA);
        row_geo(L, wi0 + kRPW, x, xn, yBl, t0, t1, t2, BBl);
    }
    __device__ __forceinline__ void us(int r, float wx, float wy, float wz, float& u,
                                       float& s) const {
        const float t = fmaf(y[r], wy, wz);
        u = fxrn[r] * fmaf(-xi[r], t, wx);      // b1.w / dmu
        s = rinv[r] * fmaf(x, wx, t);           // <eta, w>
    }
    __device__ __forceinline__ float v(int r, float wx, float wy, float wz) const {
        (void)wx;
        return B[r] * fmaf(-y[r], wz, wy);
    }
    __device__ __forceinline__ float v_above(float wx, float wy, float wz) const {
        (void)wx;
        return BA * fmaf(-yA, wz, wy);
    }
    __device__ __forceinline__ float v_below(float wx, float wy, float wz) const {
        (void)wx;
        return BBl * fmaf(-yBl, wz, wy);
    }
    __device__ __forceinline__ float s(int r, float wx, float wy, float wz) const {
        return rinv[r] * fmaf(x, wx, fmaf(y[r], wy, wz));
    }
    __device__ __forceinline__ void eta(int r, float& ex, float& ey, float& ez) const {
        ex = x * rinv[r];
        ey = y[r] * rinv[r];
        ez = rinv[r];
    }
    // tangent frame: b1 = (e_x - eta eta_x)/q, b2 = (0, eta_z, -eta_y)/q with q = sqrt(1 - eta_x^2)
    __device__ __forceinline__ void frame(int r, float (&e)[3], float (&b1)[3], float (&b2)[3],
                                          float& dmu, float& idmu) const {
        eta(r, e[0], e[1], e[2]);
        const float q = __builtin_amdgcn_sqrtf(fmaf(y[r], y[r], 1.0f)) * rinv[r];
        const float iq = __builtin_amdgcn_rcpf(q);
        b1[0] = q;
        b1[1] = -e[0] * e[1] * iq;
        b1[2] = -e[0] * e[2] * iq;
        b2[0] = 0.0f;
        b2[1] = e[2] * iq;
        b2[2] = -e[1] * iq;
        dmu = q * __builtin_amdgcn_rcpf(fxrn[r]);
        idmu = fxrn[r] * iq;
    }
};

// General grid of unit directions: per pixel b1/dmu, b2/dmu and eta from the level's geometry
// table (9 planes, written at set-up from the caller's grid).  Rows outside the level read the
// nearest row (clamped), lanes outside it column 0: their values only reach pixels outside the
// valid band.
struct GridRows {
    static constexpr bool kB2xZero = false;
    float g1[kRPW][3], g2[kRPW][3], e[kRPW][3];
    float g2A[3], g2B[3];
    __device__ __forceinline__ void load(ConstLevelDev& L, int wi0, int j) {
        const int jc = clampi(j, 0, L.cols - 1);
        const size_t plane = (size_t)L.rows * L.gpitch;
#pragma unroll
        for (int r = 0; r < kRPW; ++r) {
            const size_t o = (size_t)clampi(wi0 + r, 0, L.rows - 1) * L.gpitch + jc;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                g1[r][k] = L.geo[k * plane + o];
                g2[r][k] = L.geo[(3 + k) * plane + o];
                e[r][k] = L.geo[(6 + k) * plane + o];
            }
        }
        const size_t oA = (size_t)clampi(wi0 - 1, 0, L.rows - 1) * L.gpitch + jc;
        const size_t oB = (size_t)clampi(wi0 + kRPW, 0, L.rows - 1) * L.gpitch + jc;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            g2A[k] = L.geo[(3 + k) * plane + oA];
            g2B[k] = L.geo[(3 + k) * plane + oB];
        }
    }
    __device__ __forceinline__ void us(int r, float wx, float wy, float wz, float& u,
                                       float& s_) const {
        u = fmaf(g1[r][0], wx, fmaf(g1[r][1], wy, g1[r][2] * wz));
        s_ = fmaf(e[r][0], wx, fmaf(e[r][1], wy, e[r][2] * wz));
    }
    __device__ __forceinline__ float v(int r, float wx, float wy, float wz) const {
        return fmaf(g2[r][0], wx, fmaf(g2[r][1], wy, g2[r][2] * wz));
    }
    __device__ __forceinline__ float v_above(float wx, float wy, float wz) const {
        return fmaf(g2A[0], wx, fmaf(g2A[1], wy, g2A[2] * wz));
    }
    __device__ __forceinline__ float v_below(float wx, float wy, float wz) const {
        return fmaf(g2B[0], wx, fmaf(g2B[1], wy, g2B[2] * wz));
    }
    __device__ __forceinline__ float s(int r, float wx, float wy, float wz) const {
        return fmaf(e[r][0], wx, fmaf(e[r][1], wy, e[r][2] * wz));
    }
    __device__ __forceinline__ void eta(int r, float& ex, float& ey, float& ez) const {
        ex = e[r][0];
        ey = e[r][1];
        ez = e[r][2];
    }
    // |b1/dmu| = 1/dmu; b1, b2 are the table's vectors times dmu
    __device__ __forceinline__ void frame(int r, float (&ee)[3], float (&b1)[3], float (&b2)[3],
                                          float& dmu, float& idmu) const {
        eta(r, ee[0], ee[1], ee[2]);
        const float n2 = fmaf(g1[r][0], g1[r][0], fmaf(g1[r][1], g1[r][1], g1[r][2] * g1[r][2]));
        dmu = rsqrtf(n2);
        idmu = n2 * dmu;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            b1[k] = g1[r][k] * dmu;
            b2[k] = g2[r][k] * dmu;
        }
    }
};

// One column (beta_1) half-step of every row held by this wave.  Rows outside the image or
// outside the band still valid after the previous steps are stepped too (their values are
// finite and reach only rows that leave the valid band themselves), so every field is updated
// in place with no per-row branch.
template <int NF, bool BORDER, class G>
__device__ __forceinline__ void column_pass(float (&F)[kRPW][NF], const G& geo, bool at_left,
                                            bool at_right, float dt, float lim, float dtsig,
                                            bool dom_lit) {
#pragma unroll
    for (int r = 0; r < kRPW; ++r) {
        const float wx = F[r][0], wy = F[r][1], wz = F[r][2];
        float u, s;
        geo.us(r, wx, wy, wz, u, s);                          // b1.w / dmu, <eta, w>
        const float um = nb_prev<BORDER>(u, at_left);
        const float up = nb_next<BORDER>(u, at_right);
        const bool larger_next = fabsf(up) > fabsf(um);
        float uh = dom_lit ? (larger_next ? um : up) : (larger_next ? up : um);
        uh = __builtin_amdgcn_fmed3f(uh, -lim, lim);         // stability bound (lim = N or inf)
        // upwind step f - dt (u_hat D f + sigma s f) with D the one-sided difference toward
        // the upwind side, written as k0 f + ap f_left - am f_right with ap = dt max(u_hat, 0),
        // am = dt min(u_hat, 0), k0 = 1 - dt sigma s - ap + am (no source term for the image).
        // At the image border the missing neighbour equals the pixel itself, so its weight
        // moves into k0, i.e. the coefficient is dropped.  Per field: the left neighbour's
        // product (a multiply with the lane shift folded in), k0 f added by fmac, the right
        // neighbour's by fmac with the lane shift (3 instructions per field).
        const float du = dt * uh;
        float ap = fmaxf(du, 0.0f), am = fminf(du, 0.0f);
        if (BORDER) {
            ap = at_left ? 0.0f : ap;
            am = at_right ? 0.0f : am;
        }
        const float c = fmaf(-dtsig, s, 1.0f);
        // one of ap, am is 0, so c - (ap - am) = (c - ap) + am exactly; ap - am = |du| unless
        // a coefficient was dropped at the border
        const float d = BORDER ? ap - am : fabsf(du);
        const float k0 = c - d;
        const float k1 = 1.0f - d;
        float acc[NF];
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            const float f = F[r][k];
            const float kk = (NF == 8 && k == 7) ? k1 : k0;
            acc[k] = fmaf(kk, f, dpp_prev(f) * ap);
        }
        fmac_next_neg<NF>(acc, F[r], am);
#pragma unroll
        for (int k = 0; k < NF; ++k) F[r][k] = acc[k];
    }
}

// One row (beta_2) half-step of every row held by this wave: row neighbours from the wave's
// own registers and, for its first and last rows, the rows above and below the strip (from
// the neighbouring waves).  Same upwind form as the column pass; at the image's first and last
// row the missing neighbour's coefficient is dropped.
template <int NF, bool TOP, class G>
__device__ __forceinline__ void row_pass(float (&F)[kRPW][NF], const float (&above)[NF],
                                         const float (&below)[NF], const G& geo, int wi0, int R,
                                         float dt, float lim, float dtsig, bool dom_lit) {
    constexpr int RPW = kRPW;
    float v[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) v[r] = geo.v(r, F[r][0], F[r][1], F[r][2]);
    const float vA = geo.v_above(above[0], above[1], above[2]);
    const float vB = geo.v_below(below[0], below[1], below[2]);
    float prev[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) prev[k] = above[k];
    float vprev = vA;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int i = wi0 + r;
        float cur[NF];
#pragma unroll
        for (int k = 0; k < NF; ++k) cur[k] = F[r][k];
        const float vc = v[r];
        const bool top_b = i == 0, bot_b = i == R - 1;
        const float vm = top_b ? vc : vprev;
        const float vp = bot_b ? vc : (r + 1 < RPW ? v[r + 1 < RPW ? r + 1 : r] : vB);
        const bool larger_next = fabsf(vp) > fabsf(vm);
        float vh = dom_lit ? (larger_next ? vm : vp) : (larger_next ? vp : vm);
        vh = __builtin_amdgcn_fmed3f(vh, -lim, lim);
        const float s = geo.s(r, cur[0], cur[1], cur[2]);
        const float dv = dt * vh;
        const float ap = top_b ? 0.0f : fmaxf(dv, 0.0f);
        const float am = bot_b ? 0.0f : fminf(dv, 0.0f);
        const float c = fmaf(-dtsig, s, 1.0f);
        const float d = ap - am;          // one of ap, am is 0: c - d = (c - ap) + am exactly
        const float k0 = c - d;
        const float k1 = 1.0f - d;
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            const float fm = prev[k];
            const float fp = r + 1 < RPW ? F[r + 1 < RPW ? r + 1 : r][k] : below[k];
            const float kk = (!TOP && k == 7) ? k1 : k0;
            F[r][k] = fmaf(-am, fp, fmaf(ap, fm, kk * cur[k]));
        }
#pragma unroll
        for (int k = 0; k < NF; ++k) prev[k] = cur[k];
        vprev = vc;
    }
}

// Inertial source terms of eq:hflow_conservation that eq:assumption drops, as an explicit step
// of length dt after each column/row step of the prediction: with the camera's angular velocity
// Omega, its rate of change dOmega and linear acceleration a (uniform; rad/frame, rad/frame^2
// and 1/frame^2),
//   w  += dt (-2 Omega x w - Omega x (Omega x eta) - dOmega x eta - rho a)
//   dw += dt (-2 Omega x dw)                               (lower levels: the linear part)
// where Omega x (Omega x eta) = Omega (Omega . eta) - eta |Omega|^2, the acceleration enters
// with -rho a (from w = -Omega x eta - rho v and eq:camvel_dot), and -dOmega x eta is what a
// changing rate adds to the derivative of -Omega x eta (the paper takes Omega constant).
template <int NF, bool TOP, class G>
__device__ __forceinline__ void inertial_step(float (&F)[kRPW][NF], const G& geo, float dt,
                                              const Inertial& m) {
    constexpr int KR = TOP ? 3 : 6;
    const float oo = fmaf(m.ox, m.ox, fmaf(m.oy, m.oy, m.oz * m.oz));
    const float m2 = -2.0f * dt;
#pragma unroll
    for (int r = 0; r < kRPW; ++r) {
        float ex, ey, ez;
        geo.eta(r, ex, ey, ez);
        const float c = fmaf(m.ox, ex, fmaf(m.oy, ey, m.oz * ez));     // Omega . eta
        const float rho = F[r][KR];
        const float wx = F[r][0], wy = F[r][1], wz = F[r][2];
        // -Omega x (Omega x eta) - dOmega x eta - rho a, per component
        const float px = fmaf(m.dy, ez, fmaf(-m.dz, ey, rho * m.ax));   // (dOmega x eta) + rho a
        const float py = fmaf(m.dz, ex, fmaf(-m.dx, ez, rho * m.ay));
        const float pz = fmaf(m.dx, ey, fmaf(-m.dy, ex, rho * m.az));
        const float qx = fmaf(ex, oo, -fmaf(m.ox, c, px));
        const float qy = fmaf(ey, oo, -fmaf(m.oy, c, py));
        const float qz = fmaf(ez, oo, -fmaf(m.oz, c, pz));
        F[r][0] = fmaf(m2, fmaf(m.oy, wz, -m.oz * wy), fmaf(dt, qx, wx));
        F[r][1] = fmaf(m2, fmaf(m.oz, wx, -m.ox * wz), fmaf(dt, qy, wy));
        F[r][2] = fmaf(m2, fmaf(m.ox, wy, -m.oy * wx), fmaf(dt, qz, wz));
        if constexpr (!TOP) {
            const float dx = F[r][3], dy = F[r][4], dz = F[r][5];
            F[r][3] = fmaf(m2, fmaf(m.oy, dz, -m.oz * dy), dx);
            F[r][4] = fmaf(m2, fmaf(m.oz, dx, -m.ox * dz), dy);
            F[r][5] = fmaf(m2, fmaf(m.ox, dy, -m.oy * dx), dz);
        }
    }
}

// Sum of the 5 column neighbours j-2..j+2 of a row held across the wave's lanes; at the image's
// left/right border the border pixel repeats.  BORDER is false for regions that touch neither.
template <bool BORDER>
__device__ __forceinline__ float hsum5(float v0, bool left_b, bool right_b) {
    float m1, m2, p1, p2;
    if (BORDER) {
        m1 = clamp_prev(v0, left_b);
        m2 = clamp_prev(m1, left_b);
        p1 = clamp_next(v0, right_b);
        p2 = clamp_next(p1, right_b);
    } else {
        m1 = dpp_prev(v0);
        m2 = dpp_prev(m1);
        p1 = dpp_next(v0);
        p2 = dpp_next(p1);
    }
    return (((m2 + m1) + v0) + p1) + p2;
}

// N_s passes of the 5x5 average (1/25) of fields KX..KX+2, every row of the wave's strip (rows
// outside the band that is still valid stay finite and reach only rows that leave the band).
// A pass: horizontal sums by lane shifts, written to an LDS plane; after one barrier the
// vertical sums take the strip's own rows from registers and the two rows above and below it
// from the plane, unless the strip lies within 2 rows of the image's top or bottom, where all
// five rows are read from the plane at clamped image rows.  The planes (LDS planes 2-4 and
// 5-7, clear of the image-model planes 0-1 still read by slower waves) alternate between
// passes, so one barrier per pass suffices.
template <int NF, int KX, bool BORDER>
__device__ __forceinline__ void smooth_passes(float (&F)[kRPW][NF], float* lds, int Ns, int wave,
                                              int lane, int wi0, int gi0, int R, bool left_b,
                                              bool right_b) {
    constexpr int RPW = kRPW;
    const bool inner = wi0 - 2 >= 0 && wi0 + RPW + 2 <= R;    // wave-uniform
    for (int sp = 0; sp < Ns; ++sp) {
        float* PT = lds + (2 + 3 * (sp & 1)) * (kRegion * 64);   // [3][64 rows][64 lanes]
        float hs[RPW][3];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int row = wave * RPW + r;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                hs[r][k] = hsum5<BORDER>(F[r][KX + k], left_b, right_b);
                PT[(k * kRegion + row) * 64 + lane] = hs[r][k];
            }
        }
        __syncthreads();
        if (inner) {
            const int ra = max(wave * RPW - 2, 0), rb = min(wave * RPW + RPW, kRegion - 2);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float h[RPW + 4];
                h[0] = PT[(k * kRegion + ra) * 64 + lane];
                h[1] = PT[(k * kRegion + ra + 1) * 64 + lane];
#pragma unroll
                for (int r = 0; r < RPW; ++r) h[r + 2] = hs[r][k];
                h[RPW + 2] = PT[(k * kRegion + rb) * 64 + lane];
                h[RPW + 3] = PT[(k * kRegion + rb + 1) * 64 + lane];
#pragma unroll
                for (int r = 0; r < RPW; ++r)
                    F[r][KX + k] = ((((h[r] + h[r + 1]) + h[r + 2]) + h[r + 3]) + h[r + 4]) * 0.04f;
            }
        } else {
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int i = wi0 + r;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    float t = 0.0f;
#pragma unroll
                    for (int aa = -2; aa <= 2; ++aa) {
                        const int rr = clampi(clampi(i + aa, 0, R - 1) - gi0, 0, kRegion - 1);
                        t += PT[(k * kRegion + rr) * 64 + lane];
                    }
                    F[r][KX + k] = t * 0.04f;
                }
            }
        }
    }
}

template <typename T, bool TOP, bool IMU, class G>
__device__ __forceinline__ void level_tile(const StepArgs& a, ConstLevelDev& L, int h, int t,
                                           float* lds) {
    constexpr int NF = TOP ? 4 : 8;   // top: w(3), rho; lower: w(3), dw(3), rho, Yhat
    constexpr int NW = kNW;
    constexpr int RPW = kRPW;
    constexpr int KR = TOP ? 3 : 6;   // index of rho among the fields
    const int R = L.rows, C = L.cols;
    const int ty = t / L.tiles_x;
    const int tx = t - ty * L.tiles_x;
    const int ti0 = ty * L.th, tj0 = tx * L.tw;
    const int ti1 = min(ti0 + L.th, R), tj1 = min(tj0 + L.tw, C);
    const int halo = L.halo;
    const int gi0 = ti0 - halo, gj0 = tj0 - halo;
    const int RH = L.th + 2 * halo, RW = L.tw + 2 * halo;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
    const int par = a.parity;
    const int wi0 = gi0 + wave * RPW;             // image row of this wave's register row 0
    const int j = gj0 + lane;                     // image column of this lane
    const bool lane_ok = lane < RW && j >= 0 && j < C;
    const bool at_left = j == 0, at_right = j == C - 1;
    const bool border = gj0 <= 0 || gj0 + RW >= C;   // the region holds an image column border
    const bool left_b = border && at_left, right_b = border && at_right;
    // rows of the region held by this wave that lie in the image
    const int vi0 = max(gi0, 0), vi1 = min(gi0 + RH, R);

    // ---- geometry of this lane's pixels and of the rows just above and below the strip -------
    G geo;
    geo.load(L, wi0, j);

    // ---- load the frame-k state of the region into registers ------------------------------
    // Every load is issued unconditionally, from an address clamped into the plane (pixel 0 for
    // lanes and rows outside the image), so that all of them are in flight together; those
    // lanes and rows are zeroed afterwards.
    float F[RPW][NF];
    bool rok[RPW];
    size_t gof[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int i = wi0 + r;
        rok[r] = lane_ok && i >= vi0 && i < vi1;
        gof[r] = rok[r] ? (size_t)i * L.pitch + j : 0;
    }
    if (!L.pass_first) {    // a later pass of a split prediction: the fields after the last one
#pragma unroll
        for (int r = 0; r < RPW; ++r)
#pragma unroll
            for (int k = 0; k < NF; ++k) F[r][k] = L.mid_in[k][gof[r]];
    } else {
        const float fs = flow_in_scale<T>(L) * a.in.scale[L.stream];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const size_t g = gof[r];
#pragma unroll
            for (int k = 0; k < 3; ++k) F[r][k] = ldv((const T*)L.w[par][k], g) * fs;
            F[r][KR] = ldv((const T*)L.rho[par], g);
            if constexpr (!TOP) {
#pragma unroll
                for (int k = 0; k < 3; ++k) F[r][3 + k] = ldv((const T*)L.dw[par][k], g) * fs;
                F[r][7] = ldv((const T*)L.Y[par], g);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int k = 0; k < NF; ++k) F[r][k] = rok[r] ? F[r][k] : 0.0f;

    // ---- measurements of the update, loaded now so that their latency hides behind the
    // prediction: the new image at this wave's rows, the inverse depth at its rows and the rows
    // just above and below (clamped to the image; lanes outside it read column 0 and are
    // zeroed) -------------------------------------------------------------------------------
    const T* Ymeas = (const T*)(h == 0 ? a.in.Y[L.stream] : L.Ym[a.in.mbuf]);
    const T* Rmeas = (const T*)(h == 0 ? a.in.R[L.stream] : L.Rm[a.in.mbuf]);
    const int mp = h == 0 ? C : L.pitch;
    float ypre[RPW], rpre[RPW + 2];
    if (L.pass_last) {
        const int jc = lane_ok ? j : 0;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int i = wi0 + r;
            const float y = ldv(Ymeas, (size_t)clampi(i, 0, R - 1) * mp + jc);
            ypre[r] = (lane_ok && i >= 0 && i < R) ? y : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < RPW + 2; ++t) {
            const float rv = ldv(Rmeas, (size_t)clampi(wi0 - 1 + t, 0, R - 1) * mp + jc);
            rpre[t] = lane_ok ? rv : 0.0f;
        }
    } else {
#pragma unroll
        for (int r = 0; r < RPW; ++r) ypre[r] = 0.0f;
#pragma unroll
        for (int t = 0; t < RPW + 2; ++t) rpre[t] = 0.0f;
    }

    // ---- prediction -------------------------------------------------------------------------
    const int N = L.N;                 // the level's steps: time step 1/N, stability bound N
    const float dt = 1.0f / (float)N;
    const float fN = (float)N;
    const float sig = (L.flags & SF_READ_SOURCE_LITERAL) ? 1.0f : 0.5f;
    const float dtsig = dt * sig;
    const bool dom_lit = (L.flags & SF_READ_DOMINANT_LITERAL) != 0;
    const bool cfl = (L.flags & SF_READ_NO_CFL_CLAMP) == 0;
    const float lim = cfl ? fN : __builtin_inff();   // bound of the dominant flow
    float* XB = lds;   // [2][NW][2][NF][64] boundary rows of every wave, double-buffered

    for (int n = 0; n < L.pass_n; ++n) {   // the steps of this pass
        // column half-step: neighbours from adjacent lanes
        if (border)
            column_pass<NF, true>(F, geo, at_left, at_right, dt, lim, dtsig, dom_lit);
        else
            column_pass<NF, false>(F, geo, at_left, at_right, dt, lim, dtsig, dom_lit);
        // row half-step: neighbours from the rows above/below, across waves through LDS
        float* xb = XB + (n & 1) * (NW * 2 * NF * 64);
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            xb[((wave * 2 + 0) * NF + k) * 64 + lane] = F[0][k];
            xb[((wave * 2 + 1) * NF + k) * 64 + lane] = F[RPW - 1][k];
        }
        __syncthreads();
        // the first and last waves read a row of their own instead of the missing one: region
        // edge rows are never valid after a step, only finite
        float above[NF], below[NF];
        const int wa = wave > 0 ? wave - 1 : 0, wb = wave < NW - 1 ? wave + 1 : NW - 1;
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            above[k] = xb[((wa * 2 + 1) * NF + k) * 64 + lane];
            below[k] = xb[((wb * 2 + 0) * NF + k) * 64 + lane];
        }
        row_pass<NF, TOP>(F, above, below, geo, wi0, R, dt, lim, dtsig, dom_lit);
        if constexpr (IMU) inertial_step<NF, TOP>(F, geo, dt, a.imu[L.stream]);
    }
    __syncthreads();   // the LDS below is reused for the update phase

    if (!L.pass_last) {   // an earlier pass of a split prediction: hand the fields on
        const bool tcol = j >= tj0 && j < tj1 && lane < RW;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int i = wi0 + r;
            if (i < ti0 || i >= ti1 || !tcol) continue;
            const size_t g = (size_t)i * L.pitch + j;
#pragma unroll
            for (int k = 0; k < NF; ++k) L.mid_out[k][g] = F[r][k];
        }
        return;
    }

    // ---- update -------------------------------------------------------------------------------
    const int Ns = L.Ns;
    const int si0 = max(ti0 - 2 * Ns, 0), si1 = min(ti1 + 2 * Ns, R);
    const int sj0 = max(tj0 - 2 * Ns, 0), sj1 = min(tj1 + 2 * Ns, C);
    const int mi0 = max(si0 - 2, 0), mi1 = min(si1 + 2, R);
    float* PHG = lds;                    // [64 rows][64 lanes]
    float* PHD = lds + kRegion * 64;

    // horizontal taps of the image model in registers
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int i = wi0 + r;
        if (i < mi0 || i >= mi1) continue;           // wave-uniform
        const float y = ypre[r];
        const float ym1 = clamp_prev(y, left_b);
        const float ym2 = clamp_prev(ym1, left_b);
        const float yp1 = clamp_next(y, right_b);
        const float yp2 = clamp_next(yp1, right_b);
        float hg = 0.0f, hd = 0.0f;
        hg = fmaf(0.0625f, ym2, hg);
        hg = fmaf(0.25f, ym1, hg);
        hg = fmaf(0.375f, y, hg);
        hg = fmaf(0.25f, yp1, hg);
        hg = fmaf(0.0625f, yp2, hg);
        hd = fmaf(-0.125f, ym2, hd);
        hd = fmaf(-0.25f, ym1, hd);
        hd = fmaf(0.25f, yp1, hd);
        hd = fmaf(0.125f, yp2, hd);
        const int row = wave * RPW + r;
        PHG[row * 64 + lane] = hg;
        PHD[row * 64 + lane] = hd;
    }
    __syncthreads();

    // column neighbours of the inverse depth (clamped at the image's left/right border)
    float rleft[RPW], rright[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        rleft[r] = clamp_prev(rpre[r + 1], left_b);
        rright[r] = clamp_next(rpre[r + 1], right_b);
    }

    // vertical taps, depth model and the least-squares solve, per pixel
    {
        const float sg3 = L.g3;
        T* Yout = (T*)L.Y[1 - par];
        T* Rout = (T*)L.rho[1 - par];
        const T* Yold = (const T*)L.Y[par];
        const T* Rold = (const T*)L.rho[par];
        const bool scol = lane < RW && j >= sj0 && j < sj1;
        const bool tcol = j >= tj0 && j < tj1 && lane < RW;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int i = wi0 + r;
            if (i < si0 || i >= si1) continue;       // wave-uniform
            if (!scol) continue;
            float Yh = 0.0f, d1 = 0.0f, d2 = 0.0f;
#pragma unroll
            for (int aa = -2; aa <= 2; ++aa) {
                const int rr = (clampi(i + aa, 0, R - 1) - gi0) * 64 + lane;
                const float hg = PHG[rr], hd = PHD[rr];
                Yh = fmaf(gtap(aa), hg, Yh);
                d1 = fmaf(gtap(aa), hd, d1);
                d2 = fmaf(gtap(aa) * (float)aa, hg, d2);
            }
            const float rc = rpre[r + 1];
            const bool rv = !isnan(rc);
            float r1 = 0.0f, r2 = 0.0f;
            if (rv) {
                r1 = minabs_diff(rc, rright[r], rleft[r]);
                r2 = minabs_diff(rc, rpre[r + 2], rpre[r]);
            }
            // tangent basis and spacing at (i, j)
            float ee[3], b1[3], b2[3], dmu, idmu;
            geo.frame(r, ee, b1, b2, dmu, idmu);
            const float ex = ee[0], ey = ee[1], ez = ee[2];
            // 2-D gradients to 3-D: B (d1, d2) (b2's x component is 0 on a pinhole grid)
            const float aYx = G::kB2xZero ? b1[0] * d1 : fmaf(b1[0], d1, b2[0] * d2);
            const float aYy = fmaf(b1[1], d1, b2[1] * d2), aYz = fmaf(b1[2], d1, b2[2] * d2);
            float aRx = 0.0f, aRy = 0.0f, aRz = 0.0f, cR = 0.0f;
            const size_t gs = (size_t)i * L.pitch + j;
            const float rprior = TOP ? ldv(Rold, gs) : F[r][KR];
            const float Yprior = TOP ? ldv(Yold, gs) : F[r][7 % NF];
            if (rv) {
                const float kk = dmu * rc;
                aRx = fmaf(kk, ex, G::kB2xZero ? b1[0] * r1 : fmaf(b1[0], r1, b2[0] * r2));
                aRy = fmaf(kk, ey, fmaf(b1[1], r1, b2[1] * r2));
                aRz = fmaf(kk, ez, fmaf(b1[2], r1, b2[2] * r2));
                cR = rc - rprior;
            }
            const float cY = Yh - Yprior;
            constexpr int KX = TOP ? 0 : 3;
            const float x0 = F[r][KX] * idmu, y0 = F[r][KX + 1] * idmu, z0 = F[r][KX + 2] * idmu;
            const float dmu2 = dmu * dmu;
            const float G1 = L.g1 * dmu2;
            const float G2 = rv ? L.g2 * dmu2 : 0.0f;
            const float res1 = cY + fmaf(aYx, x0, fmaf(aYy, y0, aYz * z0));
            const float res2 = cR + fmaf(aRx, x0, fmaf(aRy, y0, aRz * z0));
            const float aa2 = fmaf(aYx, aYx, fmaf(aYy, aYy, aYz * aYz));
            const float bb = fmaf(aRx, aRx, fmaf(aRy, aRy, aRz * aRz));
            const float ab = fmaf(aYx, aRx, fmaf(aYy, aRy, aYz * aRz));
            const float cx_ = aYy * aRz - aYz * aRy, cy_ = aYz * aRx - aYx * aRz,
                        cz_ = aYx * aRy - aYy * aRx;
            const float cross2 = fmaf(cx_, cx_, fmaf(cy_, cy_, cz_ * cz_));   // aa bb - ab^2
            const float det = fmaf(sg3, sg3 + G1 * aa2 + G2 * bb, G1 * G2 * cross2);
            const float idet = __builtin_amdgcn_rcpf(det);   // det >= gamma_3^2 > 0
            const float al = -G1 * fmaf(res1, sg3, G2 * (res1 * bb - ab * res2)) * idet;
            const float be = -G2 * fmaf(res2, sg3, G1 * (res2 * aa2 - ab * res1)) * idet;
            const float rpred = F[r][KR];
            const float px0 = F[r][KX], py0 = F[r][KX + 1], pz0 = F[r][KX + 2];
            F[r][KX] = fmaf(al, aYx, fmaf(be, aRx, x0)) * dmu;
            F[r][KX + 1] = fmaf(al, aYy, fmaf(be, aRy, y0)) * dmu;
            F[r][KX + 2] = fmaf(al, aYz, fmaf(be, aRz, z0)) * dmu;
            if (i >= ti0 && i < ti1 && tcol) {
                const float rn = rv ? (L.g4 * rc + L.g5 * rpred) * __builtin_amdgcn_rcpf(L.g4 + L.g5)
                                    : rpred;
                stv(Rout, gs, rn);
                stv(Yout, gs, Yh);
                if (L.learned) {
                    // inputs of the learned update, its prior, the least-squares solution and
                    // the cost terms that judge the network's answer
                    float* lb = L.lbuf + L.lbase + (size_t)(i * C + j);
                    const size_t P = (size_t)L.ltotal;
                    // the network's input, packed as its first layer reads it
                    const uint32_t h0 = to_bf16(Yprior - 0.5f), h1 = to_bf16(Yh - 0.5f);
                    const uint32_t h2 = to_bf16(rv ? 4.0f * rc : 0.0f), h3 = to_bf16(x0 * 0.25f);
                    const uint32_t h4 = to_bf16(y0 * 0.25f), h5 = to_bf16(z0 * 0.25f);
                    const uint32_t h6 = to_bf16(F[r][KX] * idmu * 0.25f);
                    const uint32_t h7 = to_bf16(F[r][KX + 1] * idmu * 0.25f);
                    const uint32_t h8 = to_bf16(F[r][KX + 2] * idmu * 0.25f);
                    uint4* pk = reinterpret_cast<uint4*>(L.lpack + ((size_t)L.lbase + i * C + j) * 16);
                    pk[0] = make_uint4(h0 | (h1 << 16), h2 | (h3 << 16), h4 | (h5 << 16),
                                       h6 | (h7 << 16));
                    pk[1] = make_uint4(h8, 0u, 0u, 0u);
                    lb[(kLearnX0 + 0) * P] = px0;
                    lb[(kLearnX0 + 1) * P] = py0;
                    lb[(kLearnX0 + 2) * P] = pz0;
                    lb[(kLearnXP + 0) * P] = F[r][KX];
                    lb[(kLearnXP + 1) * P] = F[r][KX + 1];
                    lb[(kLearnXP + 2) * P] = F[r][KX + 2];
                    lb[(kLearnFB + 0) * P] = aYx;
                    lb[(kLearnFB + 1) * P] = aYy;
                    lb[(kLearnFB + 2) * P] = aYz;
                    lb[(kLearnFB + 3) * P] = aRx;
                    lb[(kLearnFB + 4) * P] = aRy;
                    lb[(kLearnFB + 5) * P] = aRz;
                    lb[(kLearnFB + 6) * P] = G1;
                    lb[(kLearnFB + 7) * P] = G2;
                }
            }
        }
    }

    // the learned update chooses, smooths and stores this level's flow in its own kernel
    if (L.learned) return;

    // ---- smoothing: N_s passes of the 5x5 average ---------------------------------------------
    constexpr int KX = TOP ? 0 : 3;
    if (border)
        smooth_passes<NF, KX, true>(F, lds, Ns, wave, lane, wi0, gi0, R, left_b, right_b);
    else
        smooth_passes<NF, KX, false>(F, lds, Ns, wave, lane, wi0, gi0, R, left_b, right_b);

    // ---- store the solved field of the tile -----------------------------------------------
    {
        const float os = flow_out_scale<T>(L);
        const bool tcol = j >= tj0 && j < tj1 && lane < RW;
        bool bad = false;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int i = wi0 + r;
            if (i < ti0 || i >= ti1 || !tcol) continue;
            const size_t go = (size_t)i * L.pitch + j;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T* dst = (T*)(TOP ? L.w[1 - par][k] : L.dw[1 - par][k]);
                const float v = F[r][KX + k] * os;
                bad = bad || !(fabsf(v) <= stored_max<T>());
                stv(dst, go, v);
            }
        }
        flag_nonfinite(bad, lane, L);
    }
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup w runs on XCD w mod 8), and
// each XCD has its own L2.  Hand out tiles in groups of G consecutive ones per XCD instead
// (G = min(32, n / 8)), so that neighbouring tiles, which read overlapping halos, mostly share
// an L2 while the XCDs still alternate over the grid; a bijection of [0, n), the identity on
// the tail that does not fill a whole round of groups.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_local_block(int w, int n) {
    const int g = min(32, n / kXcds);
    if (g == 0) return w;
    const int full = n / (kXcds * g) * (kXcds * g);
    if (w >= full) return w;
    const int x = w % kXcds, k = w / kXcds;      // k-th workgroup dispatched to XCD x
    return ((k / g) * kXcds + x) * g + k % g;
}

template <typename T, bool IMU, class G>
__global__ void __launch_bounds__(kBlock) k_step(StepArgs a) {
    extern __shared__ float lds[];
    const int b = xcd_local_block(blockIdx.x, gridDim.x);
    // the entry owning this block: the last one whose first block is <= b
    int lo = 0, hi = a.nent - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (level_block0(a.lv, mid) <= b) lo = mid; else hi = mid - 1;
    }
    ConstLevelDev& L = level_entry(a.lv, lo);
    if (L.top)
        level_tile<T, true, IMU, G>(a, L, L.level, b - L.block0, lds);
    else
        level_tile<T, false, IMU, G>(a, L, L.level, b - L.block0, lds);
}

// The entry and pixel of a per-pixel launch; false past the entry's last pixel.
__device__ __forceinline__ bool elem_pixel(const ElemArgs& a, int& k, int& e, int& i, int& j) {
    const int b = blockIdx.x;
    k = 0;
    while (k + 1 < a.n && a.blk[k + 1] <= b) ++k;
    e = a.ent[k];
    ConstLevelDev& L = level_entry(a.lv, e);
    const int p = (b - a.blk[k]) * kElemBlock + threadIdx.x;
    if (p >= L.rows * L.cols) return false;
    i = p / L.cols;
    j = p - i * L.cols;
    return true;
}

// ------------------------------------------------------------------------------------------
// pyramid: level h+1 = 5x5 Gaussian blur of level h sampled at (2i, 2j); inverse depth
// blurred over valid samples only (missing if none).
// ------------------------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ float rnd(float v);   // value as stored
template <> __device__ __forceinline__ float rnd<float>(float v) { return v; }
template <> __device__ __forceinline__ float rnd<__half>(float v) {
    return __half2float(__float2half(v));
}

// The entry (and its slot k in the launch) and tile of a two-level tile launch.
__device__ __forceinline__ int tile_entry(const ElemArgs& a, int& k, int& t) {
    const int b = blockIdx.x;
    k = 0;
    while (k + 1 < a.n && a.blk[k + 1] <= b) ++k;
    t = b - a.blk[k];
    return a.ent[k];
}

// One pyramid sample of a level from the level below it; `ld(ii, jj, y, r)` reads the finer
// level at (ii, jj), already clamped.  Both phases of k_pyramid use it, so a level computed in
// LDS and one read from memory are summed in the same order.
template <class Load>
__device__ __forceinline__ void pyr_sample(Load ld, int i, int j, int rows, int cols, float& y,
                                           float& r) {
    float acc = 0.0f, num = 0.0f, den = 0.0f;
#pragma unroll
    for (int aa = -2; aa <= 2; ++aa) {
        const int ii = clampi(2 * i + aa, 0, rows - 1);
#pragma unroll
        for (int bb = -2; bb <= 2; ++bb) {
            const float w = gtap(aa) * gtap(bb);
            float ys, rs;
            ld(ii, clampi(2 * j + bb, 0, cols - 1), ys, rs);
            acc = fmaf(w, ys, acc);
            if (!isnan(rs)) {
                num = fmaf(w, rs, num);
                den += w;
            }
        }
    }
    y = acc;
    r = den > 0.0f ? num / den : __int_as_float(0x7fc00000);
}

// Two pyramid levels per launch: the entry is level d (>= 1).  A block owns a TILE x TILE
// tile of level d (TILE = 16, or 32 for launches large enough to fill the chip with the bigger
// tiles) and, if level d + 1 exists, the TILE/2 x TILE/2 tile of level d + 1 above it.  The
// level d - 1 pixels the tile reads (at most 2 (TILE + 3) + 3 per side) are staged in LDS
// first, each loaded once with all of a thread's loads in flight together.  Phase 1 computes
// level d on the tile plus the rows and columns that level d + 1 reads (at most TILE + 3 per
// side) into LDS, as stored (rounded to T), and writes the tile's own pixels; phase 2 computes
// level d + 1 from LDS.  Every level-d pixel is written by exactly one block.
constexpr int kPyrThreads = 512;
template <typename T, int TILE>
__global__ void __launch_bounds__(kPyrThreads) k_pyramid(ElemArgs a) {
    constexpr int P = TILE + 3, Q = 2 * P + 3;
    constexpr int NL = (Q * Q + kPyrThreads - 1) / kPyrThreads;   // staged pixels per thread
    constexpr int NP = (P * P + kPyrThreads - 1) / kPyrThreads;   // patch pixels per thread
    constexpr int H2 = TILE / 2;
    static_assert(H2 * H2 <= kPyrThreads, "one level d + 1 pixel per thread");
    __shared__ float pY[P][P + 1], pR[P][P + 1];
    __shared__ float sY[Q][Q + 1], sR[Q][Q + 1];
    int k, t;
    const int e = tile_entry(a, k, t);
    // a stream's entries are consecutive, finest first: the finer level is entry e - 1, the
    // coarser one (if any) e + 1.  Its fields are read before knowing whether it exists (the
    // table has zeroed entries after its end), so that every table read is issued at once.
    ConstLevelDev& D = level_entry(a.lv, e);
    ConstLevelDev& S = level_entry(a.lv, e - 1);
    ConstLevelDev& U = level_entry(a.lv, e + 1);
    const int urows = U.rows, ucols = U.cols, upitch = U.pitch;
    const int mb = a.in.mbuf;
    T* const uYm = (T*)U.Ym[mb];
    T* const uRm = (T*)U.Rm[mb];
    const int ntx = (D.cols + TILE - 1) / TILE;
    const int ti0 = (t / ntx) * TILE, tj0 = (t % ntx) * TILE;
    const bool two = D.parent >= 0;
    int r0 = ti0, r1 = min(ti0 + TILE, D.rows), q0 = tj0, q1 = min(tj0 + TILE, D.cols);
    int a2 = 0, b2 = 0, c2 = 0, d2 = 0;
    if (two) {
        a2 = ti0 / 2;
        b2 = min(a2 + H2, urows);
        c2 = tj0 / 2;
        d2 = min(c2 + H2, ucols);
        r0 = min(r0, max(2 * a2 - 2, 0));
        r1 = max(r1, min(2 * b2 + 1, D.rows));
        q0 = min(q0, max(2 * c2 - 2, 0));
        q1 = max(q1, min(2 * d2 + 1, D.cols));
    }
    const int nr = r1 - r0, nc = q1 - q0;
    const bool fin = S.level == 0;
    const T* Ys = (const T*)(fin ? a.in.Y[D.stream] : S.Ym[mb]);
    const T* Rs = (const T*)(fin ? a.in.R[D.stream] : S.Rm[mb]);
    const int sp = fin ? S.cols : S.pitch;
    const int p = threadIdx.x;
    // the finer level's rows [s0, s0 + ns) and columns [u0, u0 + nu): every clamped tap
    const int s0 = max(2 * r0 - 2, 0), ns = min(2 * r1 + 1, S.rows) - s0;
    const int u0 = max(2 * q0 - 2, 0), nu = min(2 * q1 + 1, S.cols) - u0;
    {
        float vy[NL], vr[NL];
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int q = p + m * kPyrThreads;
            const int qq = q < ns * nu ? q : 0;
            const size_t idx = (size_t)(s0 + qq / nu) * sp + u0 + qq % nu;
            vy[m] = ldv(Ys, idx);
            vr[m] = ldv(Rs, idx);
        }
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int q = p + m * kPyrThreads;
            if (q < ns * nu) {
                sY[q / nu][q % nu] = vy[m];
                sR[q / nu][q % nu] = vr[m];
            }
        }
    }
    __syncthreads();
    auto from_src = [&](int ii, int jj, float& y, float& r) {
        y = sY[ii - s0][jj - u0];
        r = sR[ii - s0][jj - u0];
    };
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const int q = p + m * kPyrThreads;
        if (q >= nr * nc) continue;
        const int li = q / nc, lj = q - li * nc;
        const int i = r0 + li, j = q0 + lj;
        float y, r;
        pyr_sample(from_src, i, j, S.rows, S.cols, y, r);
        pY[li][lj] = rnd<T>(y);
        pR[li][lj] = rnd<T>(r);
        if (i >= ti0 && i < ti0 + TILE && j >= tj0 && j < tj0 + TILE) {
            stv((T*)D.Ym[mb], (size_t)i * D.pitch + j, y);
            stv((T*)D.Rm[mb], (size_t)i * D.pitch + j, r);
        }
    }
    if (!two) return;
    __syncthreads();
    const int i = a2 + p / H2, j = c2 + p % H2;
    if (p >= H2 * H2 || i >= b2 || j >= d2) return;
    auto from_lds = [&](int ii, int jj, float& y, float& r) {
        y = pY[ii - r0][jj - q0];
        r = pR[ii - r0][jj - q0];
    };
    float y, r;
    pyr_sample(from_lds, i, j, D.rows, D.cols, y, r);
    stv(uYm, (size_t)i * upitch + j, y);
    stv(uRm, (size_t)i * upitch + j, r);
}

// first frame: Yhat = G * Y, rho = measured (0 where missing), w = dw = 0, into state[0]
template <typename T>
__global__ void __launch_bounds__(kElemBlock) k_init(ElemArgs a) {
    int k0, e, i, j;
    if (!elem_pixel(a, k0, e, i, j)) return;
    ConstLevelDev& L = level_entry(a.lv, e);
    const bool fin = L.level == 0;
    const T* Ym = (const T*)(fin ? a.in.Y[L.stream] : L.Ym[a.in.mbuf]);
    const T* Rm = (const T*)(fin ? a.in.R[L.stream] : L.Rm[a.in.mbuf]);
    const int mp = fin ? L.cols : L.pitch;
    // same separable order of operations as the image model of k_step, so that a static
    // scene reproduces Yhat bit for bit
    float acc = 0.0f;
#pragma unroll
    for (int aa = -2; aa <= 2; ++aa) {
        const size_t row = (size_t)clampi(i + aa, 0, L.rows - 1) * mp;
        float hg = 0.0f;
#pragma unroll
        for (int bb = -2; bb <= 2; ++bb)
            hg = fmaf(gtap(bb), ldv(Ym, row + clampi(j + bb, 0, L.cols - 1)), hg);
        acc = fmaf(gtap(aa), hg, acc);
    }
    const size_t go = (size_t)i * L.pitch + j;
    const float r = ldv(Rm, (size_t)i * mp + j);
    stv((T*)L.Y[0], go, acc);
    stv((T*)L.rho[0], go, isnan(r) ? 0.0f : r);
    for (int k = 0; k < 3; ++k) {
        stv((T*)L.w[0][k], go, 0.0f);
        if (!L.top) stv((T*)L.dw[0][k], go, 0.0f);
        if (L.learned) L.lbuf[L.lbase + (size_t)(kLearnCorr + k) * L.ltotal + (size_t)i * L.cols + j] = 0.0f;
    }
}

// One output pixel of a stream's finest level from its flow (rad/frame, as stored): the kind
// a.kind into the planes a.outs[k] of launch slot k.  The learned update's correction is added
// here.
__device__ __forceinline__ void emit_flow(const ElemArgs& a, int k, ConstLevelDev& L, int i,
                                          int j, float wx, float wy, float wz) {
    float* out = a.outs[k];
    const size_t plane = (size_t)L.rows * L.cols;
    const size_t o = (size_t)i * L.cols + j;
    if (L.learned) {   // the learned update's correction of the output
        const float* lb = L.lbuf + L.lbase + o;
        const size_t P = (size_t)L.ltotal;
        wx += lb[kLearnCorr * P];
        wy += lb[(kLearnCorr + 1) * P];
        wz += lb[(kLearnCorr + 2) * P];
    }
    if (a.kind == SF_FLOW_W_RAD_S || a.kind == SF_FLOW_W_FRAME) {
        const float m = a.kind == SF_FLOW_W_RAD_S ? a.inv_dts[k] : 1.0f;
        out[o] = wx * m;
        out[o + plane] = wy * m;
        out[o + 2 * plane] = wz * m;
        return;
    }
    if (L.geo) {   // general grid: (b1.w, b2.w) / dmu and <eta, w> / dmu from the table
        const size_t gp = (size_t)L.rows * L.gpitch, go = (size_t)i * L.gpitch + j;
        const float* G = L.geo + go;
        if (a.kind == SF_FLOW_TANGENT_PX) {
            out[o] = fmaf(G[0], wx, fmaf(G[gp], wy, G[2 * gp] * wz));
            out[o + plane] = fmaf(G[3 * gp], wx, fmaf(G[4 * gp], wy, G[5 * gp] * wz));
        } else {
            const float n2 = fmaf(G[0], G[0], fmaf(G[gp], G[gp], G[2 * gp] * G[2 * gp]));
            out[o] = fmaf(G[6 * gp], wx, fmaf(G[7 * gp], wy, G[8 * gp] * wz)) * sqrtf(n2);
        }
        return;
    }
    const Geo g = pixel_geo(L, i, j);
    if (a.kind == SF_FLOW_TANGENT_PX) {
        out[o] = flow_u(g, wx, wy, wz);
        out[o + plane] = flow_v(g, wx, wy, wz);
    } else {   // normal: <eta, w> / dmu with dmu = sqrt(1 - eta_x^2) / (fx |r_n|)
        const float q2 = sqrtf(fmaf(g.y, g.y, 1.0f)) * g.rinv;
        out[o] = normal_s(g, wx, wy, wz) * g.fxrn / q2;
    }
}

// reconstruction w_h = bilinear(w_{h+1}) at (i/2, j/2) + dw_h, in state[parity]
// Bilinear sample of the coarser level at fine pixel (i, j); `W(ii, jj)` reads it as stored.
// The four coarse samples (i0|i1, j0|j1) and their weights.
struct Bilerp {
    int i0, i1, j0, j1;
    float w00, w01, w10, w11;
};
__device__ __forceinline__ Bilerp bilerp_at(int i, int j, int urows, int ucols) {
    Bilerp b;
    b.i0 = i >> 1;
    b.j0 = j >> 1;
    b.i1 = min(b.i0 + 1, urows - 1);
    b.j1 = min(b.j0 + 1, ucols - 1);
    const float fi = (i & 1) ? 0.5f : 0.0f, fj = (j & 1) ? 0.5f : 0.0f;
    b.w00 = (1.0f - fi) * (1.0f - fj);
    b.w01 = (1.0f - fi) * fj;
    b.w10 = fi * (1.0f - fj);
    b.w11 = fi * fj;
    return b;
}
__device__ __forceinline__ float bilerp_sum(const Bilerp& b, float v00, float v01, float v10,
                                            float v11) {
    return b.w00 * v00 + b.w01 * v01 + b.w10 * v10 + b.w11 * v11;
}

// Two reconstruction levels per launch: the entry is level h, U its parent.  A block owns a
// TILE x TILE tile of level h (TILE = 16: one pixel per thread; 32: four, for launches large
// enough to fill the chip with the bigger tiles).  Phase 1 holds U on the tile's footprint (at
// most TILE/2 + 1 per side) in LDS, as stored: reconstructed from U's parent when U is not the
// top level (the block then also writes the U pixels (i, j) with (2i, 2j) in its tile, so
// every U pixel is written once), read from the state otherwise.  Phase 2 reconstructs level h
// and, for the launch slots whose a.outs is set, writes their stream's output (emit_flow),
// bitwise what k_output would write after this launch.
template <typename T, int TILE>
__global__ void __launch_bounds__(kElemBlock) k_reconstruct(ElemArgs a) {
    constexpr int P = TILE / 2 + 1;
    constexpr int NPX = TILE * TILE / kElemBlock;                  // level-h pixels per thread
    constexpr int NPP = (P * P + kElemBlock - 1) / kElemBlock;     // footprint pixels per thread
    __shared__ float pw[3][P][P + 1];
    int slot, t;
    const int e = tile_entry(a, slot, t);
    // a stream's entries are consecutive, finest first: U = e + 1 always exists here, its
    // parent V = e + 2 only below the top (else the next stream's first level or a zeroed pad
    // entry, read but not used), so that every table read is issued at once
    ConstLevelDev& L = level_entry(a.lv, e);
    ConstLevelDev& U = level_entry(a.lv, e + 1);
    ConstLevelDev& V = level_entry(a.lv, e + 2);
    const int q = a.parity;
    const bool utop = U.top != 0;
    const int vrows = V.rows, vcols = V.cols, vpitch = V.pitch;
    const T* const vw[3] = {(const T*)V.w[q][0], (const T*)V.w[q][1], (const T*)V.w[q][2]};
    const float vin = flow_in_scale<T>(V);
    const int ntx = (L.cols + TILE - 1) / TILE;
    const int ti0 = (t / ntx) * TILE, tj0 = (t % ntx) * TILE;
    const int ti1 = min(ti0 + TILE, L.rows), tj1 = min(tj0 + TILE, L.cols);
    const int pa = ti0 >> 1, pb = min(((ti1 - 1) >> 1) + 2, U.rows);
    const int pc = tj0 >> 1, pd = min(((tj1 - 1) >> 1) + 2, U.cols);
    const int np = (pb - pa) * (pd - pc);
    // the level-h pixels of this thread (threadIdx.x + 256 m), their increments loaded before
    // the barrier
    float d[NPX][3];
#pragma unroll
    for (int m = 0; m < NPX; ++m) {
        const int px = threadIdx.x + kElemBlock * m;
        const int i = ti0 + px / TILE, j = tj0 + px % TILE;
        const size_t go = (size_t)i * L.pitch + j;
#pragma unroll
        for (int k = 0; k < 3; ++k) d[m][k] = 0.0f;
        if (i < ti1 && j < tj1)
#pragma unroll
            for (int k = 0; k < 3; ++k) d[m][k] = ldv((const T*)L.dw[q][k], go);
    }
    if (utop) {
#pragma unroll
        for (int m = 0; m < NPP; ++m) {
            const int pp = threadIdx.x + kElemBlock * m;
            if (pp >= np) continue;
            const int ui = pa + pp / (pd - pc), uj = pc + pp % (pd - pc);
            const size_t uo = (size_t)ui * U.pitch + uj;
            for (int k = 0; k < 3; ++k) pw[k][ui - pa][uj - pc] = ldv((const T*)U.w[q][k], uo);
        }
    } else {
        // every load first (the stores below may alias them for all the compiler knows);
        // footprint pixels past np load pixel (pa, pc) and are dropped
        Bilerp bv[NPP];
        float s00[NPP][3], s01[NPP][3], s10[NPP][3], s11[NPP][3], du[NPP][3];
#pragma unroll
        for (int m = 0; m < NPP; ++m) {
            const int pp = threadIdx.x + kElemBlock * m;
            const int ppc = pp < np ? pp : 0;
            const int ui = pa + ppc / (pd - pc), uj = pc + ppc % (pd - pc);
            const size_t uo = (size_t)ui * U.pitch + uj;
            bv[m] = bilerp_at(ui, uj, vrows, vcols);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                s00[m][k] = ldv(vw[k], (size_t)bv[m].i0 * vpitch + bv[m].j0);
                s01[m][k] = ldv(vw[k], (size_t)bv[m].i0 * vpitch + bv[m].j1);
                s10[m][k] = ldv(vw[k], (size_t)bv[m].i1 * vpitch + bv[m].j0);
                s11[m][k] = ldv(vw[k], (size_t)bv[m].i1 * vpitch + bv[m].j1);
                du[m][k] = ldv((const T*)U.dw[q][k], uo);
            }
        }
        const float uin = flow_in_scale<T>(U);
        const float uout = flow_out_scale<T>(U);
#pragma unroll
        for (int m = 0; m < NPP; ++m) {
            const int pp = threadIdx.x + kElemBlock * m;
            if (pp >= np) continue;
            const int ui = pa + pp / (pd - pc), uj = pc + pp % (pd - pc);
            const size_t uo = (size_t)ui * U.pitch + uj;
            const bool wr = 2 * ui >= ti0 && 2 * ui < ti1 && 2 * uj >= tj0 && 2 * uj < tj1;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float c = bilerp_sum(bv[m], s00[m][k], s01[m][k], s10[m][k], s11[m][k]);
                const float v = (c * vin + du[m][k] * uin) * uout;
                pw[k][ui - pa][uj - pc] = rnd<T>(v);
                if (wr) stv((T*)U.w[q][k], uo, v);
            }
        }
    }
    __syncthreads();
    const float uin = flow_in_scale<T>(U);
    const float lin = flow_in_scale<T>(L);
    const float lout = flow_out_scale<T>(L);
#pragma unroll
    for (int m = 0; m < NPX; ++m) {
        const int px = threadIdx.x + kElemBlock * m;
        const int i = ti0 + px / TILE, j = tj0 + px % TILE;
        if (i >= ti1 || j >= tj1) continue;
        const size_t go = (size_t)i * L.pitch + j;
        const Bilerp bu = bilerp_at(i, j, U.rows, U.cols);
        float w[3];
        for (int k = 0; k < 3; ++k) {
            const float c = bilerp_sum(bu, pw[k][bu.i0 - pa][bu.j0 - pc],
                                       pw[k][bu.i0 - pa][bu.j1 - pc],
                                       pw[k][bu.i1 - pa][bu.j0 - pc],
                                       pw[k][bu.i1 - pa][bu.j1 - pc]);
            const float v = c * uin + d[m][k] * lin;
            stv((T*)L.w[q][k], go, v * lout);
            w[k] = rnd<T>(v * lout) * lin;    // as k_output reads it back
        }
        if (a.outs[slot]) emit_flow(a, slot, L, i, j, w[0], w[1], w[2]);
    }
}

// finest-level outputs of the streams of the launch (entries with a.outs set)
template <typename T>
__global__ void __launch_bounds__(kElemBlock) k_output(ElemArgs a) {
    int k, e, i, j;
    if (!elem_pixel(a, k, e, i, j)) return;
    ConstLevelDev& L = level_entry(a.lv, e);
    const int q = a.parity;
    const size_t go = (size_t)i * L.pitch + j;
    if (a.kind == SF_FLOW_RHO) {
        a.outs[k][(size_t)i * L.cols + j] = ldv((const T*)L.rho[q], go);
        return;
    }
    const float fs = flow_in_scale<T>(L);
    emit_flow(a, k, L, i, j, ldv((const T*)L.w[q][0], go) * fs, ldv((const T*)L.w[q][1], go) * fs,
              ldv((const T*)L.w[q][2], go) * fs);
}

// ------------------------------------------------------------------------------------------
// learned update, one launch: per 16 x 42 tile of a stream's finest level, the network
// (nettile::net_tile, bitwise the per-layer launches) and then, with its output still in LDS,
// the level's N_s passes of 5x5 averaging of the least-squares solution x_ls (same order of
// operations as in k_step) and the state store, as in the plain update; then, per pixel, the
// network's correction dmu * c of the output flow, kept unless its least-squares cost
// G1 (aY.c)^2 + G2 (aR.c)^2 + g3 |c|^2 exceeds the threshold (or is not finite).  The
// correction is applied to the output (k_output, k_reconstruct), not fed back into the state.
// The averaging region is the tile plus a halo of 2 N_s (N_s <= 4), in the LDS the network
// has finished with.
// ------------------------------------------------------------------------------------------
constexpr int kCombPlane = (nettile::kNetTH + 16) * (nettile::kNetTW + 16);
static_assert((3 * nettile::kNetTH * nettile::kNetTW + 2 * 3 * kCombPlane) * sizeof(float) <=
              nettile::kNetLds, "the averaging region fits in the network's LDS");

template <typename T>
__global__ void __launch_bounds__(nettile::kNetThreads) k_net_combine(NetCombineArgs a) {
    using namespace nettile;
    constexpr int TH = kNetTH, TW = kNetTW, NT = kNetThreads;
    extern __shared__ uint2 net_lds[];
    __shared__ unsigned int nfb;
    const int b = blockIdx.x;
    int k = 0;
    while (k + 1 < a.net.segs.n && a.net.tblk[k + 1] <= b) ++k;
    ConstLevelDev& L = level_entry(a.lv, a.ent[k]);
    const int R = L.rows, C = L.cols;
    const int t = b - a.net.tblk[k];
    const int tilesx = (C + TW - 1) / TW;
    const int ti0 = (t / tilesx) * TH, tj0 = (t % tilesx) * TW;
    const int ti1 = min(ti0 + TH, R), tj1 = min(tj0 + TW, C);
    if (threadIdx.x == 0) nfb = 0;
    net_tile(a.net.in, a.net.w, a.net.bias, a.net.segs.base[k], R, C, ti0, tj0, net_lds);
    const float* out32 = reinterpret_cast<const float*>(net_lds);   // [3][TH][TW]
    float* const X = reinterpret_cast<float*>(net_lds) + 3 * TH * TW;
    float* const TM = X + 3 * kCombPlane;
    const int Ns = L.Ns;
    const int hal = 2 * Ns;
    const int gi0 = ti0 - hal, gj0 = tj0 - hal;
    const int RW = TW + 2 * hal;
    const int vi0 = max(gi0, 0), vi1 = min(ti1 + hal, R);
    const int vj0 = max(gj0, 0), vj1 = min(tj1 + hal, C);
    const size_t P = (size_t)L.ltotal;
    float* lb = L.lbuf + L.lbase;
    // the averaging region is at most TW + 16 <= 64 columns wide (N_s <= 4): a lane per column,
    // the waves take its rows in turn (no per-element division)
    static_assert(TW + 16 <= 64, "one lane per column of the averaging region");
    constexpr int NWV = NT / 64;
    const int lc = threadIdx.x & 63, lw = threadIdx.x >> 6;
    for (int i = vi0 + lw; vj0 + lc < vj1 && i < vi1; i += NWV) {
        const int j = vj0 + lc;
        const size_t p = (size_t)i * C + j;
        const int li = (i - gi0) * RW + (j - gj0);
        for (int c = 0; c < 3; ++c) X[c * kCombPlane + li] = lb[(kLearnXP + c) * P + p];
    }
    // the cost terms of this thread's tile pixels, loaded now so that their latency hides
    // behind the averaging (tile pixel q = threadIdx.x + NT m)
    constexpr int kPer = (TH * TW + NT - 1) / NT;
    const int tw = tj1 - tj0, npx = (ti1 - ti0) * tw;
    float pre[kPer][11];
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
        const int q = threadIdx.x + NT * m;
        const int qq = q < npx ? q : 0;
        const int qi = qq / tw, qj = qq % tw;
        const size_t p = (size_t)(ti0 + qi) * C + tj0 + qj;
#pragma unroll
        for (int c = 0; c < 3; ++c) pre[m][c] = out32[(c * TH + qi) * TW + qj];
#pragma unroll
        for (int c = 0; c < 8; ++c) pre[m][3 + c] = lb[(kLearnFB + c) * P + p];
    }
    __syncthreads();
    for (int sp = 1; sp <= Ns; ++sp) {
        const int rad = 2 * (Ns - sp);
        const int oi0 = max(ti0 - rad, 0), oi1 = min(ti1 + rad, R);
        const int oj0 = max(tj0 - rad, 0), oj1 = min(tj1 + rad, C);
        const int ii0 = max(oi0 - 2, 0), ii1 = min(oi1 + 2, R);
        for (int i = ii0 + lw; oj0 + lc < oj1 && i < ii1; i += NWV) {
            const int j = oj0 + lc;
            const int row = (i - gi0) * RW - gj0;
            for (int c = 0; c < 3; ++c) {
                const float* Xc = X + c * kCombPlane;
                const float m2 = Xc[row + clampi(j - 2, 0, C - 1)];
                const float m1 = Xc[row + clampi(j - 1, 0, C - 1)];
                const float v0 = Xc[row + j];
                const float p1 = Xc[row + clampi(j + 1, 0, C - 1)];
                const float p2 = Xc[row + clampi(j + 2, 0, C - 1)];
                TM[c * kCombPlane + (i - gi0) * RW + (j - gj0)] = (((m2 + m1) + v0) + p1) + p2;
            }
        }
        __syncthreads();
        for (int i = oi0 + lw; oj0 + lc < oj1 && i < oi1; i += NWV) {
            const int j = oj0 + lc;
            for (int c = 0; c < 3; ++c) {
                float s = 0.0f;
                for (int aa = -2; aa <= 2; ++aa)
                    s += TM[c * kCombPlane + (clampi(i + aa, 0, R - 1) - gi0) * RW + (j - gj0)];
                X[c * kCombPlane + (i - gi0) * RW + (j - gj0)] = s * 0.04f;
            }
        }
        __syncthreads();
    }
    const float os = flow_out_scale<T>(L);
    const int q2 = a.parity;
    unsigned int myfb = 0;
    bool bad = false;
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
        const int q = threadIdx.x + NT * m;
        if (q >= npx) continue;
        const int i = ti0 + q / tw;
        const int j = tj0 + q % tw;
        const size_t p = (size_t)i * C + j;
        const size_t go = (size_t)i * L.pitch + j;
        const int li = (i - gi0) * RW + (j - gj0);
        const float* d = pre[m];                      // pixels per frame
        const float* fbt = pre[m] + 3;
        const float eY = fbt[0] * d[0] + fbt[1] * d[1] + fbt[2] * d[2];
        const float eR = fbt[3] * d[0] + fbt[4] * d[1] + fbt[5] * d[2];
        const float cost = fbt[6] * eY * eY + fbt[7] * eR * eR +
                           L.g3 * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const bool fb = !(cost <= a.threshold) || !isfinite(cost);   // NaN and inf fall back
        myfb += fb ? 1u : 0u;
        const float dmu = pixel_dmu(L, i, j);
        for (int c = 0; c < 3; ++c) {
            const float xs = X[c * kCombPlane + li];
            lb[(kLearnXS + c) * P + p] = xs;
            lb[(kLearnCorr + c) * P + p] = fb ? 0.0f : dmu * d[c];
            T* dst = (T*)(L.top ? L.w[q2][c] : L.dw[q2][c]);
            const float v = xs * os;
            bad = bad || !(fabsf(v) <= stored_max<T>());
            stv(dst, go, v);
        }
    }
    flag_nonfinite(bad, threadIdx.x & 63, L);
    if (myfb) atomicAdd(&nfb, myfb);
    __syncthreads();
    if (threadIdx.x == 0 && nfb) atomicAdd(a.fallbacks, (unsigned long long)nfb);
}

template <typename T>
__global__ void __launch_bounds__(kElemBlock) k_learned_extract(ElemArgs a) {
    int k0, e, i, j;
    if (!elem_pixel(a, k0, e, i, j)) return;
    ConstLevelDev& L = level_entry(a.lv, e);
    const size_t npx = (size_t)L.rows * L.cols;
    const size_t o = (size_t)i * L.cols + j;
    const size_t P = (size_t)L.ltotal;
    const float* lb = L.lbuf + L.lbase + o;
    const uint16_t* pk = L.lpack + ((size_t)L.lbase + o) * 16;
    for (int k = 0; k < kLearnInputs; ++k)   // the network's inputs, as it reads them (BF16)
        a.out[k * npx + o] = __builtin_bit_cast(float, (uint32_t)pk[k] << 16);
    for (int k = kLearnInputs; k < kLearnFB; ++k) a.out[k * npx + o] = lb[k * P];
    for (int k = 0; k < 3; ++k) a.out[(kLearnFB + k) * npx + o] = lb[(kLearnXS + k) * P];
    float base[3] = {0.0f, 0.0f, 0.0f};
    if (!L.top) {
        ConstLevelDev& U = level_entry(a.lv, L.parent);
        const int q = a.parity;
        const int i0 = i >> 1, j0 = j >> 1;
        const int i1 = min(i0 + 1, U.rows - 1), j1 = min(j0 + 1, U.cols - 1);
        const float fi = (i & 1) ? 0.5f : 0.0f, fj = (j & 1) ? 0.5f : 0.0f;
        const float w00 = (1.0f - fi) * (1.0f - fj), w01 = (1.0f - fi) * fj;
        const float w10 = fi * (1.0f - fj), w11 = fi * fj;
        const float uin = flow_in_scale<T>(U);
        for (int k = 0; k < 3; ++k) {
            const T* W = (const T*)U.w[q][k];
            base[k] = (w00 * ldv(W, (size_t)i0 * U.pitch + j0) + w01 * ldv(W, (size_t)i0 * U.pitch + j1) +
                       w10 * ldv(W, (size_t)i1 * U.pitch + j0) + w11 * ldv(W, (size_t)i1 * U.pitch + j1)) *
                      uin;
        }
    }
    for (int k = 0; k < 3; ++k) a.out[(kLearnFB + 3 + k) * npx + o] = base[k];
    a.out[(kLearnFB + 6) * npx + o] = pixel_dmu(L, i, j);
}

// ------------------------------------------------------------------------------------------
// mapping a pinhole camera's frame onto a stream's finest grid (Section "Experimental
// Validation": the image and depth are mapped onto the grid before the filter runs).  Grid
// direction eta projects to source pixel (u, v) = (fx eta_x / eta_z + cx, fy eta_y / eta_z + cy);
// brightness is interpolated bilinearly with the source clamped to its edge; inverse depth
// bilinearly over the valid (not NaN) neighbours, missing when they carry less than half of
// the weight or the direction is more than 1e-3 px outside the image or behind the camera.
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kElemBlock) k_map(MapArgs a) {
    ConstLevelDev& L = level_entry(a.lv, a.ent);
    const int p = blockIdx.x * kElemBlock + threadIdx.x;
    if (p >= L.rows * L.cols) return;
    const int i = p / L.cols, j = p - i * L.cols;
    float ex, ey, ez;
    if (L.geo) {
        const size_t gp = (size_t)L.rows * L.gpitch, go = (size_t)i * L.gpitch + j;
        ex = L.geo[6 * gp + go];
        ey = L.geo[7 * gp + go];
        ez = L.geo[8 * gp + go];
    } else {
        const float x = fmaf((float)j, L.ifx, -L.cxn), y = fmaf((float)i, L.ify, -L.cyn);
        const float rinv = rsqrtf(fmaf(x, x, fmaf(y, y, 1.0f)));
        ex = x * rinv;
        ey = y * rinv;
        ez = rinv;
    }
    const bool ahead = ez > 0.0f;
    const float iz = ahead ? 1.0f / ez : 0.0f;
    const float u = ahead ? fmaf(a.fx, ex * iz, a.cx) : 0.0f;
    const float v = ahead ? fmaf(a.fy, ey * iz, a.cy) : 0.0f;
    const float tol = 1e-3f;
    const bool inside = ahead && u >= -tol && u <= (float)(a.cols - 1) + tol && v >= -tol &&
                        v <= (float)(a.rows - 1) + tol;
    const float uc = fminf(fmaxf(u, 0.0f), (float)(a.cols - 1));
    const float vc = fminf(fmaxf(v, 0.0f), (float)(a.rows - 1));
    const int j0 = min((int)uc, a.cols - 1), i0 = min((int)vc, a.rows - 1);
    const int j1 = min(j0 + 1, a.cols - 1), i1 = min(i0 + 1, a.rows - 1);
    const float fu = uc - (float)j0, fv = vc - (float)i0;
    const float w[4] = {(1.0f - fv) * (1.0f - fu), (1.0f - fv) * fu, fv * (1.0f - fu), fv * fu};
    const size_t o[4] = {(size_t)i0 * a.cols + j0, (size_t)i0 * a.cols + j1,
                         (size_t)i1 * a.cols + j0, (size_t)i1 * a.cols + j1};
    const T* Y = (const T*)a.Y;
    const T* R = (const T*)a.R;
    float yv = 0.0f, num = 0.0f, den = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        yv = fmaf(w[k], ldv(Y, o[k]), yv);
        const float r = ldv(R, o[k]);
        if (!isnan(r)) {
            num = fmaf(w[k], r, num);
            den += w[k];
        }
    }
    const size_t q = (size_t)p;
    stv((T*)a.Yout, q, yv);
    stv((T*)a.Rout, q, (inside && den >= 0.5f) ? num / den : __int_as_float(0x7fc00000));
}

}  // namespace

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
// every instantiation of the level step: storage x inertial terms x grid
#define SFLOW_STEP_KERNELS                                                                     \
    (const void*)k_step<float, false, PinholeRows>, (const void*)k_step<__half, false, PinholeRows>, \
    (const void*)k_step<float, true, PinholeRows>, (const void*)k_step<__half, true, PinholeRows>,   \
    (const void*)k_step<float, false, GridRows>, (const void*)k_step<__half, false, GridRows>,       \
    (const void*)k_step<float, true, GridRows>, (const void*)k_step<__half, true, GridRows>

int frame_input_kind(const void* func) {
    const void* step[] = {SFLOW_STEP_KERNELS};
    const void* pyr[] = {(const void*)k_pyramid<float, kTile2>,
                         (const void*)k_pyramid<__half, kTile2>,
                         (const void*)k_pyramid<float, 2 * kTile2>,
                         (const void*)k_pyramid<__half, 2 * kTile2>};
    for (const void* f : step)
        if (f == func) return 2;
    for (const void* f : pyr)
        if (f == func) return 1;
    return 0;
}

hipError_t prepare_kernels(size_t max_lds_bytes) {
    const void* fns[] = {SFLOW_STEP_KERNELS};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)max_lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static int elem_blocks(const ElemArgs& a) { return a.blk[a.n]; }

hipError_t launch_pyramid(int storage, int tile, const ElemArgs& a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const dim3 g(elem_blocks(a)), b(kPyrThreads);
    if (tile == 2 * kTile2) {
        if (storage == SF_FP16)
            hipLaunchKernelGGL((k_pyramid<__half, 2 * kTile2>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_pyramid<float, 2 * kTile2>), g, b, 0, s, a);
    } else {
        if (storage == SF_FP16)
            hipLaunchKernelGGL((k_pyramid<__half, kTile2>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_pyramid<float, kTile2>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_map(int storage, const MapArgs& a, int pixels, hipStream_t s) {
    const int blocks = (pixels + kElemBlock - 1) / kElemBlock;
    if (blocks == 0) return hipSuccess;
    if (storage == SF_FP16)
        hipLaunchKernelGGL(k_map<__half>, dim3(blocks), dim3(kElemBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_map<float>, dim3(blocks), dim3(kElemBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init(int storage, const ElemArgs& a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    if (storage == SF_FP16)
        hipLaunchKernelGGL(k_init<__half>, dim3(elem_blocks(a)), dim3(kElemBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(elem_blocks(a)), dim3(kElemBlock), 0, s, a);
    return hipGetLastError();
}

template <typename T, bool IMU>
static void launch_step_g(bool grid, const StepArgs& a, dim3 g, dim3 b, size_t lds,
                          hipStream_t s) {
    if (grid)
        hipLaunchKernelGGL((k_step<T, IMU, GridRows>), g, b, lds, s, a);
    else
        hipLaunchKernelGGL((k_step<T, IMU, PinholeRows>), g, b, lds, s, a);
}

hipError_t launch_step(int storage, bool inertial, bool grid, const StepArgs& a, int nblocks,
                       size_t lds, hipStream_t s) {
    const dim3 g(nblocks), b(kBlock);
    if (storage == SF_FP16) {
        if (inertial)
            launch_step_g<__half, true>(grid, a, g, b, lds, s);
        else
            launch_step_g<__half, false>(grid, a, g, b, lds, s);
    } else {
        if (inertial)
            launch_step_g<float, true>(grid, a, g, b, lds, s);
        else
            launch_step_g<float, false>(grid, a, g, b, lds, s);
    }
    return hipGetLastError();
}

hipError_t launch_reconstruct(int storage, int tile, const ElemArgs& a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const dim3 g(elem_blocks(a)), b(kElemBlock);
    if (tile == 2 * kTile2) {
        if (storage == SF_FP16)
            hipLaunchKernelGGL((k_reconstruct<__half, 2 * kTile2>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_reconstruct<float, 2 * kTile2>), g, b, 0, s, a);
    } else {
        if (storage == SF_FP16)
            hipLaunchKernelGGL((k_reconstruct<__half, kTile2>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_reconstruct<float, kTile2>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_output(int storage, const ElemArgs& a, hipStream_t s) {
    if (storage == SF_FP16)
        hipLaunchKernelGGL(k_output<__half>, dim3(elem_blocks(a)), dim3(kElemBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_output<float>, dim3(elem_blocks(a)), dim3(kElemBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace sflow

namespace sflow {
hipError_t launch_learned_extract(int storage, const ElemArgs& a, hipStream_t s) {
    if (storage == SF_FP16)
        hipLaunchKernelGGL(k_learned_extract<__half>, dim3(elem_blocks(a)), dim3(kElemBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_learned_extract<float>, dim3(elem_blocks(a)), dim3(kElemBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_net_combine(int storage, const NetCombineArgs& args, hipStream_t s) {
    using namespace nettile;
    static std::atomic<uint64_t> prepared{0};   // devices the LDS limit was raised on
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = 1ull << (dev & 63);
    if (!(prepared.load() & bit)) {
        for (const void* f : {(const void*)k_net_combine<float>, (const void*)k_net_combine<__half>}) {
            e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kNetLds);
            if (e != hipSuccess) return e;
        }
        prepared.fetch_or(bit);
    }
    NetCombineArgs a = args;
    int blocks = 0;
    for (int k = 0; k < a.net.segs.n; ++k) {
        a.net.tblk[k] = blocks;
        blocks += ((a.net.segs.rows[k] + kNetTH - 1) / kNetTH) * ((a.net.segs.cols[k] + kNetTW - 1) / kNetTW);
    }
    a.net.tblk[a.net.segs.n] = blocks;
    if (blocks == 0) return hipSuccess;
    if (storage == SF_FP16)
        hipLaunchKernelGGL(k_net_combine<__half>, dim3(blocks), dim3(kNetThreads), kNetLds, s, a);
    else
        hipLaunchKernelGGL(k_net_combine<float>, dim3(blocks), dim3(kNetThreads), kNetLds, s, a);
    return hipGetLastError();
}
}  // namespace sflow
