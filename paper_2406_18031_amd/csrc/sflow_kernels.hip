// gfx950 kernels of the structure-flow filter.
//
// k_step is the hot path: one workgroup owns one output tile of one pyramid level and runs,
// for that tile, every stage of the level's predictor-update block (Section "Filter
// Architecture") with the tile plus a halo resident in LDS:
//   prediction  N upwind column/row half-steps (Section "Numerical prediction"),
//   image model 5x5 Gaussian-weighted linear fit as separable passes (eq:img_model),
//   depth model occlusion-aware one-sided differences (eq:dominant_b1/b2),
//   update      the 3x3 least-squares system (eq:LS_update) solved in residual form
//               around the prior: x = x0 + alpha a_Y + beta a_rho (2x2 inner system),
//   smoothing   N_s passes of the 5x5 average,
//   rho update  eq:cost_invdepth.
// The halo is max(N, 2) + 2 N_s pixels per side: each half-step invalidates one pixel on
// each interior side of the region, each 5x5 pass two.  Column half-steps give every wave
// whole rows (lane = column), row half-steps whole columns (lane = row), so neighbours along
// the pass come from lane shuffles and LDS reads within the wave and only a block barrier
// separates the passes.  Geometry (unit ray, tangent basis, pixel spacing) is recomputed
// from the pinhole intrinsics in registers instead of being read from memory.
#include "sflow_internal.h"

namespace sflow {
namespace {

__device__ __forceinline__ float ldv(const float* p, size_t i) { return p[i]; }
__device__ __forceinline__ float ldv(const __half* p, size_t i) { return __half2float(p[i]); }
__device__ __forceinline__ void stv(float* p, size_t i, float v) { p[i] = v; }
__device__ __forceinline__ void stv(__half* p, size_t i, float v) { p[i] = __float2half(v); }

template <typename T> __device__ __forceinline__ float flow_in_scale(const LevelDev& L);
template <> __device__ __forceinline__ float flow_in_scale<float>(const LevelDev&) { return 1.0f; }
template <> __device__ __forceinline__ float flow_in_scale<__half>(const LevelDev& L) {
    return 1.0f / L.qscale;
}
template <typename T> __device__ __forceinline__ float flow_out_scale(const LevelDev& L);
template <> __device__ __forceinline__ float flow_out_scale<float>(const LevelDev&) { return 1.0f; }
template <> __device__ __forceinline__ float flow_out_scale<__half>(const LevelDev& L) {
    return L.qscale;
}

// 1-D Gaussian taps g = [1, 4, 6, 4, 1] / 16 (exact in binary)
__device__ __forceinline__ float gtap(int a) {
    return a == 0 ? 0.375f : ((a == 1 || a == -1) ? 0.25f : 0.0625f);
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

__device__ __forceinline__ Geo pixel_geo(const LevelDev& L, int i, int j) {
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
template <typename T, bool TOP>
__device__ __forceinline__ void level_tile(const StepArgs& a, const LevelDev& L, int h, int t,
                                           float* lds) {
    const int R = L.rows, C = L.cols;
    const int ty = t / L.tiles_x;
    const int tx = t - ty * L.tiles_x;
    const int ti0 = ty * L.th, tj0 = tx * L.tw;
    const int ti1 = min(ti0 + L.th, R), tj1 = min(tj0 + L.tw, C);
    const int halo = L.halo;
    const int gi0 = ti0 - halo, gj0 = tj0 - halo;
    const int RH = L.th + 2 * halo, RW = L.tw + 2 * halo;
    const int P = RW | 1;           // odd pitch: column passes read LDS without bank conflicts
    const int PS = RH * P;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    constexpr int NW = kBlock / 64;
    constexpr bool top = TOP;
    const int par = a.parity;
    constexpr int nf = TOP ? 4 : 8; // transported fields: w(3), rho | w(3), dw(3), rho, Y
    // plane of field k: top {w0, w1, w2, rho} -> {0, 1, 2, 3}; lower -> {0..7}
    auto plane = [&](int k) -> float* { return lds + k * PS; };
    constexpr int prho = TOP ? 3 : 6;

    const int vi0 = max(gi0, 0), vi1 = min(gi0 + RH, R);
    const int vj0 = max(gj0, 0), vj1 = min(gj0 + RW, C);

    // ---- load frame-k state of the region -----------------------------------------------
    {
        const float fs = flow_in_scale<T>(L) * a.scale;
        for (int i = vi0 + wave; i < vi1; i += NW) {
            const int j = gj0 + lane;
            if (lane < RW && j >= vj0 && j < vj1) {
                const size_t gidx = (size_t)i * L.pitch + j;
                const int li = (i - gi0) * P + lane;
#pragma unroll
                for (int k = 0; k < 3; ++k) plane(k)[li] = ldv((const T*)L.w[par][k], gidx) * fs;
                plane(prho)[li] = ldv((const T*)L.rho[par], gidx);
                if (!top) {
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        plane(3 + k)[li] = ldv((const T*)L.dw[par][k], gidx) * fs;
                    plane(7)[li] = ldv((const T*)L.Y[par], gidx);
                }
            }
        }
    }
    __syncthreads();

    // ---- prediction: N steps of column then row half-steps --------------------------------
    const int N = L.N;
    const float dt = 1.0f / (float)N;
    const float fN = (float)N;
    const float sig = (a.flags & SF_READ_SOURCE_LITERAL) ? 1.0f : 0.5f;
    const bool dom_lit = (a.flags & SF_READ_DOMINANT_LITERAL) != 0;
    const bool cfl = (a.flags & SF_READ_NO_CFL_CLAMP) == 0;
    int ci0 = vi0, ci1 = vi1, cj0 = vj0, cj1 = vj1;

    for (int n = 0; n < N; ++n) {
#pragma unroll
        for (int axis = 0; axis < 2; ++axis) {   // 0: column pass (along j), 1: row pass (along i)
            const bool colp = axis == 0;
            // the new valid interval along the pass axis shrinks on interior sides
            const int lo = colp ? cj0 : ci0, hi = colp ? cj1 : ci1;
            const int ext = colp ? C : R;
            const int nlo = lo > 0 ? lo + 1 : lo;
            const int nhi = hi < ext ? hi - 1 : hi;
            // lines orthogonal to the pass, one per wave; lane = position along the pass
            const int l0 = colp ? ci0 : cj0, l1 = colp ? ci1 : cj1;
            const int g0 = colp ? gj0 : gi0;
            const int span = colp ? RW : RH;
            const int stride = colp ? 1 : P;
            for (int line = l0 + wave; line < l1; line += NW) {
                const int pos = g0 + lane;            // image coordinate along the pass
                const bool act = lane < span && pos >= lo && pos < hi;
                const int i = colp ? line : pos;
                const int j = colp ? pos : line;
                const int base = colp ? (line - gi0) * P + lane : lane * P + (line - gj0);
                float f[8];
                float u = 0.0f;
                Geo g = {};
                if (act) {
#pragma unroll
                    for (int k = 0; k < nf; ++k) f[k] = plane(k)[base];
                    g = pixel_geo(L, i, j);
                    u = colp ? flow_u(g, f[0], f[1], f[2]) : flow_v(g, f[0], f[1], f[2]);
                }
                float um = __shfl_up(u, 1);
                float up = __shfl_down(u, 1);
                if (pos == 0) um = u;
                if (pos == ext - 1) up = u;
                const bool upd = act && pos >= nlo && pos < nhi;
                float nv[8];
                if (upd) {
                    const bool larger_next = fabsf(up) > fabsf(um);
                    float uh = dom_lit ? (larger_next ? um : up) : (larger_next ? up : um);
                    if (cfl) uh = fminf(fmaxf(uh, -fN), fN);
                    const float s = normal_s(g, f[0], f[1], f[2]);
                    const bool back = uh > 0.0f;
                    const int nb = back ? (pos > 0 ? base - stride : base)
                                        : (pos < ext - 1 ? base + stride : base);
#pragma unroll
                    for (int k = 0; k < nf; ++k) {
                        const float fn = plane(k)[nb];
                        const float D = back ? f[k] - fn : fn - f[k];
                        const float sg = (!TOP && k == 7) ? 0.0f : sig;
                        nv[k] = f[k] - dt * (uh * D + sg * f[k] * s);
                    }
                }
                wave_sync();
                if (upd) {
#pragma unroll
                    for (int k = 0; k < nf; ++k) plane(k)[base] = nv[k];
                }
                wave_sync();
            }
            __syncthreads();
            if (colp) { cj0 = nlo; cj1 = nhi; } else { ci0 = nlo; ci1 = nhi; }
        }
    }

    // ---- update ---------------------------------------------------------------------------
    const int Ns = L.Ns;
    const int si0 = max(ti0 - 2 * Ns, 0), si1 = min(ti1 + 2 * Ns, R);
    const int sj0 = max(tj0 - 2 * Ns, 0), sj1 = min(tj1 + 2 * Ns, C);
    const int mi0 = max(si0 - 2, 0), mi1 = min(si1 + 2, R);
    const int mj0 = max(sj0 - 2, 0), mj1 = min(sj1 + 2, C);
    float* YN = plane(top ? 4 : 0);
    float* HG = plane(top ? 5 : 1);
    float* HD = plane(top ? 6 : 2);
    float* X[3] = {plane(top ? 0 : 3), plane(top ? 1 : 4), plane(top ? 2 : 5)};
    const T* Ymeas = (const T*)(h == 0 ? a.Y1 : L.Ym);
    const T* Rmeas = (const T*)(h == 0 ? a.R1 : L.Rm);
    const int mp = h == 0 ? C : L.pitch;

    for (int i = mi0 + wave; i < mi1; i += NW) {
        const int j = gj0 + lane;
        if (lane < RW && j >= mj0 && j < mj1)
            YN[(i - gi0) * P + lane] = ldv(Ymeas, (size_t)i * mp + j);
    }
    __syncthreads();
    // horizontal taps of the image model: HG = g * Y, HD = (g d) * Y along j
    for (int i = mi0 + wave; i < mi1; i += NW) {
        const int j = gj0 + lane;
        if (lane < RW && j >= sj0 && j < sj1) {
            const int row = (i - gi0) * P - gj0;
            float hg = 0.0f, hd = 0.0f;
#pragma unroll
            for (int bb = -2; bb <= 2; ++bb) {
                const float y = YN[row + clampi(j + bb, 0, C - 1)];
                hg = fmaf(gtap(bb), y, hg);
                hd = fmaf(gtap(bb) * (float)bb, y, hd);
            }
            HG[(i - gi0) * P + lane] = hg;
            HD[(i - gi0) * P + lane] = hd;
        }
    }
    __syncthreads();

    {
        const float sg3 = L.g3;
        T* Yout = (T*)L.Y[1 - par];
        T* Rout = (T*)L.rho[1 - par];
        const T* Yold = (const T*)L.Y[par];
        const T* Rold = (const T*)L.rho[par];
        for (int i = si0 + wave; i < si1; i += NW) {
            const int j = gj0 + lane;
            if (!(lane < RW && j >= sj0 && j < sj1)) continue;
            const int li = (i - gi0) * P + lane;
            // brightness model: vertical taps
            float Yh = 0.0f, d1 = 0.0f, d2 = 0.0f;
#pragma unroll
            for (int aa = -2; aa <= 2; ++aa) {
                const int r = (clampi(i + aa, 0, R - 1) - gi0) * P + lane;
                const float hg = HG[r], hd = HD[r];
                Yh = fmaf(gtap(aa), hg, Yh);
                d1 = fmaf(gtap(aa), hd, d1);
                d2 = fmaf(gtap(aa) * (float)aa, hg, d2);
            }
            // depth model from the level's measured inverse depth
            const size_t gm = (size_t)i * mp;
            const float rc = ldv(Rmeas, gm + j);
            const bool rv = !isnan(rc);
            float r1 = 0.0f, r2 = 0.0f;
            if (rv) {
                r1 = minabs_diff(rc, ldv(Rmeas, gm + min(j + 1, C - 1)),
                                 ldv(Rmeas, gm + max(j - 1, 0)));
                r2 = minabs_diff(rc, ldv(Rmeas, (size_t)min(i + 1, R - 1) * mp + j),
                                 ldv(Rmeas, (size_t)max(i - 1, 0) * mp + j));
            }
            // geometry
            const Geo g = pixel_geo(L, i, j);
            const float ex = g.x * g.rinv, ey = g.y * g.rinv, ez = g.rinv;
            const float q = sqrtf(fmaf(g.y, g.y, 1.0f)) * g.rinv;    // sqrt(1 - eta_x^2)
            const float iq = 1.0f / q;
            const float b1x = q, b1y = -ex * ey * iq, b1z = -ex * ez * iq;
            const float b2y = ez * iq, b2z = -ey * iq;              // b2x = 0
            const float dmu = q / g.fxrn;
            // data terms in pixel units: E = dmu^2 (a_hat . xi + c_hat) with xi = x / dmu
            const float aYx = b1x * d1, aYy = fmaf(b1y, d1, b2y * d2), aYz = fmaf(b1z, d1, b2z * d2);
            float aRx = 0.0f, aRy = 0.0f, aRz = 0.0f, cR = 0.0f;
            const float rprior = top ? ldv(Rold, (size_t)i * L.pitch + j) : plane(prho)[li];
            const float Yprior = top ? ldv(Yold, (size_t)i * L.pitch + j) : plane(7)[li];
            if (rv) {
                const float k = dmu * rc;
                aRx = fmaf(k, ex, b1x * r1);
                aRy = fmaf(k, ey, fmaf(b1y, r1, b2y * r2));
                aRz = fmaf(k, ez, fmaf(b1z, r1, b2z * r2));
                cR = rc - rprior;
            }
            const float cY = Yh - Yprior;
            const float idmu = 1.0f / dmu;
            const float x0 = X[0][li] * idmu, y0 = X[1][li] * idmu, z0 = X[2][li] * idmu;
            const float dmu2 = dmu * dmu;
            const float G1 = L.g1 * dmu2;
            const float G2 = rv ? L.g2 * dmu2 : 0.0f;
            const float res1 = cY + fmaf(aYx, x0, fmaf(aYy, y0, aYz * z0));
            const float res2 = cR + fmaf(aRx, x0, fmaf(aRy, y0, aRz * z0));
            const float aa = fmaf(aYx, aYx, fmaf(aYy, aYy, aYz * aYz));
            const float bb = fmaf(aRx, aRx, fmaf(aRy, aRy, aRz * aRz));
            const float ab = fmaf(aYx, aRx, fmaf(aYy, aRy, aYz * aRz));
            const float cx_ = aYy * aRz - aYz * aRy, cy_ = aYz * aRx - aYx * aRz,
                        cz_ = aYx * aRy - aYy * aRx;
            const float cross2 = fmaf(cx_, cx_, fmaf(cy_, cy_, cz_ * cz_));   // aa bb - ab^2
            const float det = fmaf(sg3, sg3 + G1 * aa + G2 * bb, G1 * G2 * cross2);
            const float al = -G1 * fmaf(res1, sg3, G2 * (res1 * bb - ab * res2)) / det;
            const float be = -G2 * fmaf(res2, sg3, G1 * (res2 * aa - ab * res1)) / det;
            X[0][li] = fmaf(al, aYx, fmaf(be, aRx, x0)) * dmu;
            X[1][li] = fmaf(al, aYy, fmaf(be, aRy, y0)) * dmu;
            X[2][li] = fmaf(al, aYz, fmaf(be, aRz, z0)) * dmu;
            if (i >= ti0 && i < ti1 && j >= tj0 && j < tj1) {
                const size_t go = (size_t)i * L.pitch + j;
                const float rpred = plane(prho)[li];
                const float rn = rv ? (L.g4 * rc + L.g5 * rpred) / (L.g4 + L.g5) : rpred;
                stv(Rout, go, rn);
                stv(Yout, go, Yh);
            }
        }
    }
    __syncthreads();

    // ---- smoothing: N_s passes of the 5x5 average (separable sums, clamped borders) -------
    float* TMP[3] = {YN, HG, HD};
    for (int sp = 1; sp <= Ns; ++sp) {
        const int r = 2 * (Ns - sp);
        const int oi0 = max(ti0 - r, 0), oi1 = min(ti1 + r, R);
        const int oj0 = max(tj0 - r, 0), oj1 = min(tj1 + r, C);
        const int ii0 = max(oi0 - 2, 0), ii1 = min(oi1 + 2, R);
        for (int i = ii0 + wave; i < ii1; i += NW) {
            const int j = gj0 + lane;
            if (lane < RW && j >= oj0 && j < oj1) {
                const int row = (i - gi0) * P - gj0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    float s = 0.0f;
#pragma unroll
                    for (int bb = -2; bb <= 2; ++bb) s += X[k][row + clampi(j + bb, 0, C - 1)];
                    TMP[k][(i - gi0) * P + lane] = s;
                }
            }
        }
        __syncthreads();
        for (int i = oi0 + wave; i < oi1; i += NW) {
            const int j = gj0 + lane;
            if (lane < RW && j >= oj0 && j < oj1) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    float s = 0.0f;
#pragma unroll
                    for (int aa = -2; aa <= 2; ++aa)
                        s += TMP[k][(clampi(i + aa, 0, R - 1) - gi0) * P + lane];
                    X[k][(i - gi0) * P + lane] = s * 0.04f;
                }
            }
        }
        __syncthreads();
    }

    // ---- store the solved field of the tile -----------------------------------------------
    {
        const float os = flow_out_scale<T>(L);
        for (int i = ti0 + wave; i < ti1; i += NW) {
            const int j = tj0 + lane;
            if (lane < L.tw && j < tj1) {
                const size_t go = (size_t)i * L.pitch + j;
                const int li = (i - gi0) * P + (j - gj0);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    T* dst = (T*)(top ? L.w[1 - par][k] : L.dw[1 - par][k]);
                    stv(dst, go, X[k][li] * os);
                }
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_step(StepArgs a) {
    extern __shared__ float lds[];
    const int b = blockIdx.x;
    int h = 0;
    for (int k = 1; k < a.nlev; ++k)
        if (b >= a.lv[k].block0) h = k;
    const LevelDev& L = a.lv[h];
    if (L.top)
        level_tile<T, true>(a, L, h, b - L.block0, lds);
    else
        level_tile<T, false>(a, L, h, b - L.block0, lds);
}

// ------------------------------------------------------------------------------------------
// pyramid: level h+1 = 5x5 Gaussian blur of level h sampled at (2i, 2j); inverse depth
// blurred over valid samples only (missing if none)
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_pyramid(const T* Ys, const T* Rs, int sp, int Rsrc,
                                                 int Csrc, T* Yd, T* Rd, int dp, int Rdst,
                                                 int Cdst) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= Cdst || i >= Rdst) return;
    float acc = 0.0f, num = 0.0f, den = 0.0f;
#pragma unroll
    for (int aa = -2; aa <= 2; ++aa) {
        const size_t row = (size_t)clampi(2 * i + aa, 0, Rsrc - 1) * sp;
#pragma unroll
        for (int bb = -2; bb <= 2; ++bb) {
            const float w = gtap(aa) * gtap(bb);
            const size_t idx = row + clampi(2 * j + bb, 0, Csrc - 1);
            acc = fmaf(w, ldv(Ys, idx), acc);
            const float r = ldv(Rs, idx);
            if (!isnan(r)) {
                num = fmaf(w, r, num);
                den += w;
            }
        }
    }
    stv(Yd, (size_t)i * dp + j, acc);
    stv(Rd, (size_t)i * dp + j, den > 0.0f ? num / den : __int_as_float(0x7fc00000));
}

// first frame: Yhat = G * Y, rho = measured (0 where missing), w = dw = 0, into state[0]
template <typename T>
__global__ void __launch_bounds__(256) k_init(const LevelDev* lvp, int h, const T* Ym,
                                              const T* Rm, int mp) {
    const LevelDev& L = lvp[h];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= L.cols || i >= L.rows) return;
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
    }
}

// reconstruction w_h = bilinear(w_{h+1}) at (i/2, j/2) + dw_h, in state[q]
template <typename T>
__global__ void __launch_bounds__(256) k_reconstruct(const LevelDev* lvp, int h, int q) {
    const LevelDev& L = lvp[h];
    const LevelDev& U = lvp[h + 1];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= L.cols || i >= L.rows) return;
    const int i0 = i >> 1, j0 = j >> 1;
    const int i1 = min(i0 + 1, U.rows - 1), j1 = min(j0 + 1, U.cols - 1);
    const float fi = (i & 1) ? 0.5f : 0.0f, fj = (j & 1) ? 0.5f : 0.0f;
    const float w00 = (1.0f - fi) * (1.0f - fj), w01 = (1.0f - fi) * fj;
    const float w10 = fi * (1.0f - fj), w11 = fi * fj;
    const float uin = flow_in_scale<T>(U);
    const float lin = flow_in_scale<T>(L);
    const float lout = flow_out_scale<T>(L);
    const size_t go = (size_t)i * L.pitch + j;
    for (int k = 0; k < 3; ++k) {
        const T* W = (const T*)U.w[q][k];
        const float c = w00 * ldv(W, (size_t)i0 * U.pitch + j0) + w01 * ldv(W, (size_t)i0 * U.pitch + j1) +
                        w10 * ldv(W, (size_t)i1 * U.pitch + j0) + w11 * ldv(W, (size_t)i1 * U.pitch + j1);
        const float v = c * uin + ldv((const T*)L.dw[q][k], go) * lin;
        stv((T*)L.w[q][k], go, v * lout);
    }
}

// finest-level outputs
template <typename T>
__global__ void __launch_bounds__(256) k_output(const LevelDev* lvp, int q, int kind,
                                                float inv_dt, float* out) {
    const LevelDev& L = lvp[0];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= L.cols || i >= L.rows) return;
    const size_t go = (size_t)i * L.pitch + j;
    const size_t plane = (size_t)L.rows * L.cols;
    const size_t o = (size_t)i * L.cols + j;
    if (kind == SF_FLOW_RHO) {
        out[o] = ldv((const T*)L.rho[q], go);
        return;
    }
    const float fs = flow_in_scale<T>(L);
    const float wx = ldv((const T*)L.w[q][0], go) * fs;
    const float wy = ldv((const T*)L.w[q][1], go) * fs;
    const float wz = ldv((const T*)L.w[q][2], go) * fs;
    if (kind == SF_FLOW_W_RAD_S || kind == SF_FLOW_W_FRAME) {
        const float m = kind == SF_FLOW_W_RAD_S ? inv_dt : 1.0f;
        out[o] = wx * m;
        out[o + plane] = wy * m;
        out[o + 2 * plane] = wz * m;
        return;
    }
    const Geo g = pixel_geo(L, i, j);
    if (kind == SF_FLOW_TANGENT_PX) {
        out[o] = flow_u(g, wx, wy, wz);
        out[o + plane] = flow_v(g, wx, wy, wz);
    } else {   // normal: <eta, w> / dmu with dmu = sqrt(1 - eta_x^2) / (fx |r_n|)
        const float q2 = sqrtf(fmaf(g.y, g.y, 1.0f)) * g.rinv;
        out[o] = normal_s(g, wx, wy, wz) * g.fxrn / q2;
    }
}

}  // namespace

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
hipError_t prepare_kernels(size_t max_lds_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)k_step<float>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)max_lds_bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_step<__half>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds_bytes);
}

hipError_t launch_pyramid(int storage, const LevelDev* lv, const LevelDev*, int h,
                          const void* Ysrc, const void* Rsrc, int src_pitch, hipStream_t s) {
    const LevelDev& S = lv[h];
    const LevelDev& D = lv[h + 1];
    dim3 grid((D.cols + 255) / 256, D.rows);
    if (storage == SF_FP16)
        hipLaunchKernelGGL(k_pyramid<__half>, grid, dim3(256), 0, s, (const __half*)Ysrc,
                           (const __half*)Rsrc, src_pitch, S.rows, S.cols, (__half*)D.Ym,
                           (__half*)D.Rm, D.pitch, D.rows, D.cols);
    else
        hipLaunchKernelGGL(k_pyramid<float>, grid, dim3(256), 0, s, (const float*)Ysrc,
                           (const float*)Rsrc, src_pitch, S.rows, S.cols, (float*)D.Ym,
                           (float*)D.Rm, D.pitch, D.rows, D.cols);
    return hipGetLastError();
}

hipError_t launch_init(int storage, const LevelDev* lv, const LevelDev* lv_dev, int h,
                       const void* Ym, const void* Rm, int mp, hipStream_t s) {
    dim3 grid((lv[h].cols + 255) / 256, lv[h].rows);
    if (storage == SF_FP16)
        hipLaunchKernelGGL(k_init<__half>, grid, dim3(256), 0, s, lv_dev, h, (const __half*)Ym,
                           (const __half*)Rm, mp);
    else
        hipLaunchKernelGGL(k_init<float>, grid, dim3(256), 0, s, lv_dev, h, (const float*)Ym,
                           (const float*)Rm, mp);
    return hipGetLastError();
}

hipError_t launch_step(int storage, const StepArgs& a, int nblocks, size_t lds, hipStream_t s) {
    if (storage == SF_FP16)
        hipLaunchKernelGGL(k_step<__half>, dim3(nblocks), dim3(kBlock), lds, s, a);
    else
        hipLaunchKernelGGL(k_step<float>, dim3(nblocks), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_reconstruct(int storage, const LevelDev* lv, const LevelDev* lv_dev, int h,
                              int q, hipStream_t s) {
    dim3 grid((lv[h].cols + 255) / 256, lv[h].rows);
    if (storage == SF_FP16)
        hipLaunchKernelGGL(k_reconstruct<__half>, grid, dim3(256), 0, s, lv_dev, h, q);
    else
        hipLaunchKernelGGL(k_reconstruct<float>, grid, dim3(256), 0, s, lv_dev, h, q);
    return hipGetLastError();
}

hipError_t launch_output(int storage, const LevelDev* lv, const LevelDev* lv_dev, int q,
                         int kind, float inv_dt, float* out, hipStream_t s) {
    dim3 grid((lv[0].cols + 255) / 256, lv[0].rows);
    if (storage == SF_FP16)
        hipLaunchKernelGGL(k_output<__half>, grid, dim3(256), 0, s, lv_dev, q, kind, inv_dt, out);
    else
        hipLaunchKernelGGL(k_output<float>, grid, dim3(256), 0, s, lv_dev, q, kind, inv_dt, out);
    return hipGetLastError();
}

}  // namespace sflow
